"""ctypes binding of libavs (include/avs.h).

Argument marshalling only: every computation runs in the HIP library.
PyTorch provides the device memory (VDF region and workspace) and the HIP
stream.  Importing this module loads ``libavs.so`` from this package
directory and raises if it has not been built (``__graft_entry__.build()``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# AVS_LIBRARY selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("AVS_LIBRARY", os.path.join(_HERE, "libavs.so"))

AVS_OK, AVS_E_INVALID, AVS_E_CAPACITY, AVS_E_HIP, AVS_E_STATE, AVS_E_NUMERIC = 0, -1, -2, -3, -4, -5
AVS_FP64, AVS_FP32 = 0, 1
AVS_COPY, AVS_SPLIT, AVS_MERGE = 0, 1, 2

EXPORTS = ("avs_mu_ref_from_kn", "avs_vdf_bytes", "avs_workspace_bytes", "avs_init_mesh", "avs_step",
           "avs_moments", "avs_moments_noalloc", "avs_adapt", "avs_remap", "avs_leaves", "avs_plan", "avs_criterion",
           "avs_check", "avs_set_leaves", "avs_get_state", "avs_set_state", "avs_get_cells", "avs_profile",
           "avs_profile_read", "avs_batch_workspace_bytes", "avs_batch_create", "avs_batch_step",
           "avs_batch_check", "avs_batch_tune", "avs_batch_adapt", "avs_batch_remap", "avs_batch_destroy", "avs_mlp_param_count", "avs_mlp_state_bytes",
           "avs_mlp_create", "avs_mlp_get_params", "avs_mlp_set_params", "avs_mlp_forward", "avs_mlp_grad",
           "avs_mlp_adam", "avs_mlp_train_step", "avs_mlp_destroy", "avs_features", "avs_adapt_learned",
           "avs_auto_params", "avs_initial_avs", "avs_set_separated", "avs_implicit_bytes", "avs_step_implicit",
           "avs_rykov_equilibrium", "avs_dia_bytes", "avs_dia_create", "avs_dia_step", "avs_dia_step_implicit", "avs_dia_get_state",
           "avs_dia_adapt", "avs_dia_remap", "avs_dia_destroy", "avs_destroy", "avs_last_error")


class avs_rykov(C.Structure):
    _fields_ = [("Z_rot", C.c_double), ("delta", C.c_double), ("omega0", C.c_double), ("omega1", C.c_double)]


class avs_vspace(C.Structure):
    _fields_ = [("dim", C.c_int32), ("max_level", C.c_int32), ("base", C.c_int32 * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("leaf_capacity", C.c_int64)]


class avs_gas(C.Structure):
    _fields_ = [("R", C.c_double), ("Pr", C.c_double), ("omega", C.c_double), ("mu_ref", C.c_double),
                ("T_ref", C.c_double), ("model", C.c_int32), ("law", C.c_int32), ("C_s", C.c_double)]


class avs_pmesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("ncells", C.c_int64), ("nfaces", C.c_int64),
                ("cell_vol", C.c_void_p), ("cell_ctr", C.c_void_p), ("face_lr", C.c_void_p),
                ("face_area", C.c_void_p), ("face_nrm", C.c_void_p), ("face_ctr", C.c_void_p),
                ("face_shift", C.c_void_p), ("nbc", C.c_int32), ("bc_kind", C.c_void_p), ("bc_state", C.c_void_p)]


class avs_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("dt", C.c_double), ("venkat_K", C.c_double)]


class avs_adam(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double)]


class avs_flow(C.Structure):
    _fields_ = [("dim", C.c_int32), ("R", C.c_double), ("gamma", C.c_double), ("Ma", C.c_double),
                ("T_inf", C.c_double), ("T_wall", C.c_double), ("rho_inf", C.c_double),
                ("direction", C.c_double * 3), ("rdv_sigmas", C.c_double), ("h_std", C.c_double),
                ("separated", C.c_int32)]


class avs_auto(C.Structure):
    _fields_ = [("T0", C.c_double), ("sigma_inf", C.c_double), ("sigma_0", C.c_double), ("sigma_w", C.c_double),
                ("U_inf", C.c_double), ("centre", C.c_double * 3), ("R_dv", C.c_double), ("h_min", C.c_double),
                ("L_max", C.c_int32), ("L_w", C.c_int32), ("L_min", C.c_int32), ("L_sep", C.c_int32),
                ("C1", C.c_double), ("C2", C.c_double), ("k_sigma", C.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libavs.so not found at {LIB_PATH}: build it with __graft_entry__.build()")
    # torch's HIP runtime must be the first one in the process: a HIP runtime
    # loaded ahead of it by this library would leave torch's, or ours, without
    # a device
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, D, VP = C.POINTER, C.c_int32, C.c_int64, C.c_double, C.c_void_p
    sig = {
        "avs_mu_ref_from_kn": (D, [D, D, D, D, D, D]),
        "avs_vdf_bytes": (C.c_size_t, [P(avs_vspace), P(avs_pmesh), P(avs_opts)]),
        "avs_workspace_bytes": (C.c_size_t, [P(avs_vspace), P(avs_pmesh), P(avs_opts)]),
        "avs_init_mesh": (I32, [P(avs_vspace), P(avs_pmesh), P(avs_gas), P(avs_opts), VP, VP, C.c_size_t, VP,
                                C.c_size_t, VP, P(VP)]),
        "avs_step": (I32, [VP, I32, VP]),
        "avs_check": (I32, [VP]),
        "avs_moments": (I32, [VP, VP, VP]),
        "avs_moments_noalloc": (I32, [VP, VP, VP]),
        "avs_adapt": (I32, [VP, D, D, VP, I32, VP, P(I64)]),
        "avs_remap": (I32, [VP, I32]),
        "avs_leaves": (I32, [VP, P(I64), P(I64), VP, VP, VP, VP]),
        "avs_plan": (I32, [VP, VP, VP, VP]),
        "avs_criterion": (I32, [VP, VP]),
        "avs_set_leaves": (I32, [VP, I64, VP, VP]),
        "avs_get_state": (I32, [VP, VP, VP]),
        "avs_set_state": (I32, [VP, VP, VP]),
        "avs_get_cells": (I32, [VP, I64, VP, VP]),
        "avs_profile": (I32, [VP, I32]),
        "avs_profile_read": (I32, [VP, I32, VP, VP, VP]),
        "avs_batch_workspace_bytes": (C.c_size_t, [I32]),
        "avs_batch_create": (I32, [I32, VP, VP, C.c_size_t, P(VP)]),
        "avs_batch_step": (I32, [VP, I32, I32]),
        "avs_batch_check": (I32, [VP]),
        "avs_batch_tune": (I32, [VP, VP]),
        "avs_batch_adapt": (I32, [VP, VP, VP, VP]),
        "avs_batch_remap": (I32, [VP, I32]),
        "avs_batch_destroy": (None, [VP]),
        "avs_mlp_param_count": (I64, []),
        "avs_mlp_state_bytes": (C.c_size_t, [I64]),
        "avs_mlp_create": (I32, [VP, I64, D, D, VP, C.c_size_t, VP, P(VP)]),
        "avs_mlp_get_params": (I32, [VP, VP]),
        "avs_mlp_set_params": (I32, [VP, VP]),
        "avs_mlp_forward": (I32, [VP, VP, I64, VP]),
        "avs_mlp_grad": (I32, [VP, VP, VP, VP, I64, VP, VP]),
        "avs_mlp_adam": (I32, [VP, VP, P(avs_adam)]),
        "avs_mlp_train_step": (I32, [VP, VP, VP, VP, I64, P(avs_adam), VP]),
        "avs_mlp_destroy": (None, [VP]),
        "avs_features": (I32, [VP, VP, VP]),
        "avs_adapt_learned": (I32, [VP, VP, D, D, VP, I32, D, VP, P(I64), P(I32)]),
        "avs_auto_params": (I32, [P(avs_flow), P(avs_auto), P(avs_vspace)]),
        "avs_initial_avs": (I32, [VP, P(avs_flow), D, D, P(I64)]),
        "avs_set_separated": (I32, [VP, D, D, I32]),
        "avs_implicit_bytes": (I32, [VP, P(C.c_size_t)]),
        "avs_rykov_equilibrium": (I32, [VP, P(avs_rykov), VP, I64, VP, C.c_size_t]),
        "avs_dia_bytes": (I32, [VP, I64, P(C.c_size_t)]),
        "avs_dia_create": (I32, [VP, P(avs_rykov), VP, I64, VP, C.c_size_t, P(VP)]),
        "avs_dia_adapt": (I32, [VP, D, D, VP, I32, VP, P(I64)]),
        "avs_dia_remap": (I32, [VP]),
        "avs_dia_step": (I32, [VP, I32]),
        "avs_dia_step_implicit": (I32, [VP, I32, I32, I32]),
        "avs_dia_get_state": (I32, [VP, VP, VP]),
        "avs_dia_destroy": (None, [VP]),
        "avs_step_implicit": (I32, [VP, I32, I32, I32, VP, C.c_size_t, VP]),
        "avs_destroy": (None, [VP]),
        "avs_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


class AvsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"avs status {status}: {msg}")
        self.status = status


def _check(st):
    if st != AVS_OK:
        raise AvsError(st, lib.avs_last_error().decode())


def _ptr(a):
    return a.ctypes.data if a is not None else None


def mu_ref_from_kn(Kn, omega, R, T_ref=1.0, rho_ref=1.0, L_ref=1.0):
    return lib.avs_mu_ref_from_kn(Kn, omega, R, T_ref, rho_ref, L_ref)


def _flow(dim, R, gamma, Ma, T_inf, T_wall, rho_inf=1.0, direction=(1.0, 0.0, 0.0), rdv_sigmas=4.0, h_std=0.6,
          separated=False):
    d = tuple(float(x) for x in direction) + (0.0,) * (3 - len(direction))
    return avs_flow(int(dim), float(R), float(gamma), float(Ma), float(T_inf), float(T_wall), float(rho_inf),
                    (C.c_double * 3)(*d[:3]), float(rdv_sigmas), float(h_std), int(bool(separated)))


def auto_params(**flow):
    """Adaptive parameters of the freestream ``flow`` (keywords of avs_flow)
    and the velocity space that realises them: (params dict, vspace dict)."""
    a, v = avs_auto(), avs_vspace()
    _check(lib.avs_auto_params(C.byref(_flow(**flow)), C.byref(a), C.byref(v)))
    D = int(flow['dim'])
    params = {k: (list(getattr(a, k))[:D] if k == 'centre' else getattr(a, k)) for k, _ in avs_auto._fields_}
    vs = dict(dim=v.dim, max_level=v.max_level, base=tuple(v.base[:D]), lo=tuple(v.lo[:D]), hi=tuple(v.hi[:D]),
              leaf_capacity=v.leaf_capacity)
    return params, vs


class Case:
    """One context of the library plus the device memory it runs in."""

    def __init__(self, mesh, vspace, gas, dt, venkat_K, prim0, precision=AVS_FP64, leaf_capacity=None,
                 device="cuda:0", stream=None):
        import torch
        self._torch = torch
        D = int(mesh["dim"])
        self.dim = D
        self.P = 2 if D == 2 else 1
        self.nc = int(mesh["ncells"])
        keep = {}

        def arr(name, dtype):
            a = np.ascontiguousarray(mesh[name], dtype=dtype)
            keep[name] = a
            return a.ctypes.data
        pm = avs_pmesh()
        pm.dim = D
        pm.ncells = self.nc
        pm.nfaces = int(mesh["nfaces"])
        pm.cell_vol = arr("cell_vol", np.float64)
        pm.cell_ctr = arr("cell_ctr", np.float64)
        pm.face_lr = arr("face_lr", np.int64)
        pm.face_area = arr("face_area", np.float64)
        pm.face_nrm = arr("face_nrm", np.float64)
        pm.face_ctr = arr("face_ctr", np.float64)
        pm.face_shift = arr("face_shift", np.float64) if "face_shift" in mesh else None
        pm.nbc = int(mesh["nbc"])
        pm.bc_kind = arr("bc_kind", np.int32)
        pm.bc_state = arr("bc_state", np.float64)
        vs = avs_vspace()
        vs.dim = D
        vs.max_level = int(vspace["max_level"])
        for d in range(D):
            vs.base[d] = int(vspace["base"][d])
            vs.lo[d] = float(vspace["lo"][d])
            vs.hi[d] = float(vspace["hi"][d])
        nroot = int(np.prod([vs.base[d] for d in range(D)]))
        vs.leaf_capacity = int(leaf_capacity if leaf_capacity is not None else nroot * (2 ** D) ** vs.max_level)
        self.leaf_capacity = vs.leaf_capacity
        g = avs_gas()
        g.R, g.Pr, g.omega, g.T_ref = (float(gas[k]) for k in ("R", "Pr", "omega", "T_ref"))
        g.mu_ref = float(gas["mu_ref"]) if gas.get("mu_ref") is not None else mu_ref_from_kn(
            gas["Kn"], gas["omega"], gas["R"], gas["T_ref"], gas.get("rho_ref", 1.0), gas.get("L_ref", 1.0))
        g.model = int(gas.get("model", 1))
        g.law = int(gas.get("law", 0))           # viscosity: 0 power law, 1 Sutherland
        g.C_s = float(gas.get("C_s", 0.0))
        op = avs_opts()
        op.precision = int(precision)
        op.dt = float(dt)
        op.venkat_K = float(venkat_K)
        self.gas, self.vs, self.opts, self.pm, self._keep = g, vs, op, pm, keep
        vb = lib.avs_vdf_bytes(C.byref(vs), C.byref(pm), C.byref(op))
        wb = lib.avs_workspace_bytes(C.byref(vs), C.byref(pm), C.byref(op))
        if vb == 0 or wb == 0:
            raise AvsError(AVS_E_INVALID, lib.avs_last_error().decode())
        self.device = torch.device(device)
        self.vdf_mem = torch.empty(vb, dtype=torch.uint8, device=self.device)
        self.ws_mem = torch.empty(wb, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        p0 = np.ascontiguousarray(prim0, dtype=np.float64)
        ctx = C.c_void_p()
        _check(lib.avs_init_mesh(C.byref(vs), C.byref(pm), C.byref(g), C.byref(op), p0.ctypes.data,
                                 self.vdf_mem.data_ptr(), vb, self.ws_mem.data_ptr(), wb,
                                 self.stream.cuda_stream, C.byref(ctx)))
        self.ctx = ctx

    # -- entry points -------------------------------------------------------
    def step(self, n=1, residual=False):
        res = np.zeros(self.dim + 2) if residual else None
        _check(lib.avs_step(self.ctx, int(n), _ptr(res)))
        return res

    def step_implicit(self, n=1, macro=60, micro=2, residual=False):
        """Implicit steps (IUGKS) with ``macro`` and ``micro`` symmetric
        sweeps; the right-hand-side region is allocated once per case."""
        if getattr(self, "_imp_res", None) is None:
            nb = C.c_size_t()
            _check(lib.avs_implicit_bytes(self.ctx, C.byref(nb)))
            self._imp_res = self._torch.empty(max(nb.value, 256), dtype=self._torch.uint8, device=self.device)
        res = np.zeros(self.dim + 2) if residual else None
        _check(lib.avs_step_implicit(self.ctx, int(n), int(macro), int(micro), self._imp_res.data_ptr(),
                                     self._imp_res.numel(), _ptr(res)))
        return res

    def rykov_equilibrium(self, states, Z_rot=3.5, delta=1.0 / 1.55, omega0=0.2354, omega1=0.3049, out=None):
        """Rykov equilibrium (G, H, R) on the current leaves for states
        [n][3 + 3D] = (rho, U, T_t, T_r, q_t, q_r); returns a device tensor
        [3, n, ld] in the context's precision."""
        t = self._torch
        st = t.as_tensor(np.ascontiguousarray(states, np.float64), device=self.device)
        n = st.shape[0]
        ld = C.c_int64()
        nn = C.c_int64()
        _check(lib.avs_leaves(self.ctx, C.byref(nn), C.byref(ld), None, None, None, None))
        dt = t.float64 if self.opts.precision == AVS_FP64 else t.float32
        if out is None:
            out = t.empty((3, n, ld.value), dtype=dt, device=self.device)
        g = avs_rykov(float(Z_rot), float(delta), float(omega0), float(omega1))
        _check(lib.avs_rykov_equilibrium(self.ctx, C.byref(g), st.data_ptr(), n, out.data_ptr(),
                                         out.numel() * out.element_size()))
        t.cuda.synchronize(self.device)
        return out

    def check(self):
        """Raise AvsError if a kernel found a non-physical state since the
        context was made (waits for the stream)."""
        _check(lib.avs_check(self.ctx))

    def moments(self, fields=True, totals=True):
        f = self._torch.empty((self.nc, 2 * self.dim + 2), dtype=self._torch.float64, device=self.device) if fields else None
        t = np.zeros(self.dim + 2) if totals else None
        _check(lib.avs_moments(self.ctx, f.data_ptr() if f is not None else None, _ptr(t)))
        return f, t

    def moments_noalloc(self, fields_out=None, totals=True):
        """avs_moments through the entry point that allocates nothing (its
        partial sums live in the library's static device array); fields go
        into ``fields_out`` (a float64 device tensor [nc, 2*dim+2]) if given."""
        f = fields_out
        if f is not None and (tuple(f.shape) != (self.nc, 2 * self.dim + 2) or f.dtype != self._torch.float64
                              or not f.is_contiguous()):
            raise ValueError(f"fields_out must be a contiguous float64 tensor of shape ({self.nc}, {2 * self.dim + 2})")
        t = np.zeros(self.dim + 2) if totals else None
        _check(lib.avs_moments_noalloc(self.ctx, f.data_ptr() if f is not None else None, _ptr(t)))
        return f, t

    def adapt(self, C1, C2, probes=None, flags_out=None):
        """Plain adaptation.  Returns (effective flags as numpy, n_new); with
        ``flags_out`` (device int8 tensor of >= nleaves entries) the flags
        stay on the device and None is returned in their place."""
        n_old = self.nleaves()
        flags = flags_out if flags_out is not None else self._torch.empty(max(n_old, 1), dtype=self._torch.int8,
                                                                           device=self.device)
        pr = np.ascontiguousarray(probes, dtype=np.float64) if probes is not None else None
        nn = C.c_int64()
        _check(lib.avs_adapt(self.ctx, float(C1), float(C2), _ptr(pr), 0 if pr is None else len(pr),
                             flags.data_ptr(), C.byref(nn)))
        if flags_out is not None:
            return None, nn.value
        self._torch.cuda.synchronize(self.device)
        return flags[:n_old].cpu().numpy(), nn.value

    def features(self, mlp, out=None):
        """Feature rows of the current leaves, int16 tensor [nleaves, 32]
        holding bfloat16 bit patterns (written on this case's stream)."""
        n = self.nleaves()
        if out is None:
            out = self._torch.empty((max(n, 1), 32), dtype=self._torch.int16, device=self.device)
        _check(lib.avs_features(self.ctx, mlp.h, out.data_ptr()))
        return out[:n]

    def adapt_learned(self, mlp, C1, C2, probes=None, tail_tol=1e-4, flags_out=None):
        """Adaptation with the learned proposal; returns (flags or None, n_new, fallback)."""
        n_old = self.nleaves()
        flags = flags_out if flags_out is not None else self._torch.empty(max(n_old, 1), dtype=self._torch.int8,
                                                                           device=self.device)
        pr = np.ascontiguousarray(probes, dtype=np.float64) if probes is not None else None
        nn, fb = C.c_int64(), C.c_int32()
        _check(lib.avs_adapt_learned(self.ctx, mlp.h, float(C1), float(C2), _ptr(pr), 0 if pr is None else len(pr),
                                     float(tail_tol), flags.data_ptr(), C.byref(nn), C.byref(fb)))
        if flags_out is not None:
            return None, nn.value, bool(fb.value)
        self._torch.cuda.synchronize(self.device)
        return flags[:n_old].cpu().numpy(), nn.value, bool(fb.value)

    def remap(self, correction=2):
        _check(lib.avs_remap(self.ctx, int(correction)))

    def nleaves(self):
        n, ld = C.c_int64(), C.c_int64()
        _check(lib.avs_leaves(self.ctx, C.byref(n), C.byref(ld), None, None, None, None))
        return n.value

    def leaves(self):
        n, ld = C.c_int64(), C.c_int64()
        _check(lib.avs_leaves(self.ctx, C.byref(n), C.byref(ld), None, None, None, None))
        lev = np.zeros(n.value, np.int32)
        idx = np.zeros((n.value, self.dim), np.int32)
        xi = np.zeros((n.value, self.dim))
        w = np.zeros(n.value)
        _check(lib.avs_leaves(self.ctx, C.byref(n), C.byref(ld), lev.ctypes.data, idx.ctypes.data,
                              xi.ctypes.data, w.ctypes.data))
        return dict(n=n.value, ld=ld.value, level=lev, idx=idx, xi=xi, w=w)

    def plan(self, n_new):
        kind = np.zeros(n_new, np.int32)
        src = np.zeros(n_new, np.int64)
        child = np.zeros(n_new, np.int32)
        _check(lib.avs_plan(self.ctx, kind.ctypes.data, src.ctypes.data, child.ctypes.data))
        return kind, src, child

    def criterion(self, n_old):
        Mk = np.zeros(n_old)
        _check(lib.avs_criterion(self.ctx, Mk.ctypes.data))
        return Mk

    def initial_avs(self, C1, C2, **flow):
        """Step-0 velocity space for the freestream ``flow`` (keywords of
        avs_flow; the case must use the velocity space auto_params gives for
        it; ``separated=True`` for a flow that separates); returns the leaf
        count."""
        n = C.c_int64()
        _check(lib.avs_initial_avs(self.ctx, C.byref(_flow(**flow)), float(C1), float(C2), C.byref(n)))
        return n.value

    def set_separated(self, r_lo, r_hi, level):
        """Separated-zone floor on every later adaptation: elements centred in
        r_lo < |xi| < r_hi keep at least ``level`` (from the roots); a level
        below 0 removes it."""
        _check(lib.avs_set_separated(self.ctx, float(r_lo), float(r_hi), int(level)))

    def set_leaves(self, level, idx):
        lev = np.ascontiguousarray(level, np.int32)
        ix = np.ascontiguousarray(idx, np.int32)
        _check(lib.avs_set_leaves(self.ctx, len(lev), lev.ctypes.data, ix.ctypes.data))

    def get_state(self):
        n = self.nleaves()
        vdf = np.zeros((self.P, self.nc, n))
        W = np.zeros((self.nc, self.dim + 2))
        _check(lib.avs_get_state(self.ctx, vdf.ctypes.data, W.ctypes.data))
        return vdf, W

    def get_W(self):
        W = np.zeros((self.nc, self.dim + 2))
        _check(lib.avs_get_state(self.ctx, None, W.ctypes.data))
        return W

    def set_state(self, vdf, W):
        """vdf None: closed Maxwellian of W; W None: W = moments of vdf."""
        v = None if vdf is None else np.ascontiguousarray(vdf, np.float64)
        w = None if W is None else np.ascontiguousarray(W, np.float64)
        _check(lib.avs_set_state(self.ctx, _ptr(v), _ptr(w)))

    def get_cells(self, cells):
        c = np.ascontiguousarray(cells, np.int64)
        out = np.zeros((self.P, len(c), self.nleaves()))
        _check(lib.avs_get_cells(self.ctx, len(c), c.ctypes.data, out.ctypes.data))
        return out

    def profile(self, enable=True):
        _check(lib.avs_profile(self.ctx, 1 if enable else 0))

    def profile_read(self):
        """{kernel group: (total ms, launches)} since profiling was enabled."""
        nmax = 32
        names = C.create_string_buffer(32 * nmax)
        ms = np.zeros(nmax)
        cnt = np.zeros(nmax, np.int64)
        n = lib.avs_profile_read(self.ctx, nmax, names, ms.ctypes.data, cnt.ctypes.data)
        if n < 0:
            raise AvsError(AVS_E_STATE, lib.avs_last_error().decode())
        raw = names.raw
        return {raw[32 * i:32 * i + 32].split(b"\0")[0].decode(): (float(ms[i]), int(cnt[i])) for i in range(n)}

    def close(self):
        if getattr(self, "ctx", None):
            lib.avs_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """The learned refinement proposal's network and its device state."""

    def __init__(self, params, max_batch=16384, rho_ref=1.0, T_ref=1.0, device="cuda:0", stream=None):
        import torch
        self._torch = torch
        self.device = torch.device(device)
        self.nparam = int(lib.avs_mlp_param_count())
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.shape != (self.nparam,):
            raise AvsError(AVS_E_INVALID, f"expected {self.nparam} parameters")
        nb = lib.avs_mlp_state_bytes(int(max_batch))
        if nb == 0:
            raise AvsError(AVS_E_INVALID, lib.avs_last_error().decode())
        self.state = torch.empty(nb, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.max_batch = int(max_batch)
        h = C.c_void_p()
        _check(lib.avs_mlp_create(p.ctypes.data, int(max_batch), float(rho_ref), float(T_ref), self.state.data_ptr(),
                                  nb, self.stream.cuda_stream, C.byref(h)))
        self.h = h

    def get_params(self):
        p = np.zeros(self.nparam, np.float32)
        _check(lib.avs_mlp_get_params(self.h, p.ctypes.data))
        return p

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        _check(lib.avs_mlp_set_params(self.h, p.ctypes.data))

    def forward(self, feat, n=None):
        n = feat.shape[0] if n is None else int(n)
        out = self._torch.empty((max(n, 1), 3), dtype=self._torch.float32, device=self.device)
        _check(lib.avs_mlp_forward(self.h, feat.data_ptr(), n, out.data_ptr()))
        return out[:n]

    def grad(self, feat, flags, rows=None, n=None):
        n = (rows.shape[0] if rows is not None else feat.shape[0]) if n is None else int(n)
        g = self._torch.empty(self.nparam, dtype=self._torch.float32, device=self.device)
        loss = C.c_double()
        _check(lib.avs_mlp_grad(self.h, feat.data_ptr(), flags.data_ptr(), None if rows is None else rows.data_ptr(),
                                n, g.data_ptr(), C.byref(loss)))
        return g, loss.value

    @staticmethod
    def _hp(lr, beta1, beta2, eps):
        return avs_adam(lr=float(lr), beta1=float(beta1), beta2=float(beta2), eps=float(eps))

    def adam(self, grad, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        hp = self._hp(lr, beta1, beta2, eps)
        _check(lib.avs_mlp_adam(self.h, grad.data_ptr(), C.byref(hp)))

    def train_step(self, feat, flags, rows=None, n=None, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, loss=False):
        n = (rows.shape[0] if rows is not None else feat.shape[0]) if n is None else int(n)
        hp = self._hp(lr, beta1, beta2, eps)
        out = C.c_double()
        _check(lib.avs_mlp_train_step(self.h, feat.data_ptr(), flags.data_ptr(),
                                      None if rows is None else rows.data_ptr(), n, C.byref(hp),
                                      C.byref(out) if loss else None))
        return out.value if loss else None

    def close(self):
        if getattr(self, "h", None):
            lib.avs_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass



class Diatomic:
    """Explicit steps and adaptation of the Rykov diatomic model on a Case's
    mesh and leaves (FP64, 2-D or 3-D).  prim0 rows are (rho, U, T_t, T_r)."""

    def __init__(self, case, prim0, Z_rot=3.5, delta=1.0 / 1.55, omega0=0.2354, omega1=0.3049, max_leaves=None):
        t = case._torch
        self.case = case
        ml = int(max_leaves if max_leaves is not None else case.nleaves())
        nb = C.c_size_t()
        _check(lib.avs_dia_bytes(case.ctx, ml, C.byref(nb)))
        self.mem = t.empty(nb.value, dtype=t.uint8, device=case.device)
        p0 = np.ascontiguousarray(prim0, dtype=np.float64)
        if p0.shape != (case.nc, case.dim + 3):
            raise ValueError(f"prim0 must have shape ({case.nc}, {case.dim + 3})")
        g = avs_rykov(float(Z_rot), float(delta), float(omega0), float(omega1))
        h = C.c_void_p()
        _check(lib.avs_dia_create(case.ctx, C.byref(g), p0.ctypes.data, ml, self.mem.data_ptr(), nb.value,
                                  C.byref(h)))
        self.h = h

    def adapt(self, C1, C2, probes=None):
        """Adaptation driven by the diatomic state and the optional probe
        rows (rho, U, T) of equilibrium states; returns (flags, n_new)."""
        t = self.case._torch
        n_old = self.case.nleaves()
        flags = t.empty(max(n_old, 1), dtype=t.int8, device=self.case.device)
        nn = C.c_int64()
        pr = np.ascontiguousarray(np.atleast_2d(probes), dtype=np.float64) if probes is not None else None
        npr = 0 if pr is None else pr.shape[0]
        if pr is not None and pr.shape[1] != self.case.dim + 2:
            raise ValueError(f"probe rows must have {self.case.dim + 2} entries")
        _check(lib.avs_dia_adapt(self.h, float(C1), float(C2), None if pr is None else pr.ctypes.data, npr,
                                 flags.data_ptr(), C.byref(nn)))
        t.cuda.synchronize(self.case.device)
        return flags[:n_old].cpu().numpy(), nn.value

    def remap(self):
        _check(lib.avs_dia_remap(self.h))

    def step(self, n=1):
        _check(lib.avs_dia_step(self.h, int(n)))

    def step_implicit(self, n, n_macro, n_micro):
        """Implicit steps (the context's dt) with n_macro predictor and
        n_micro micro symmetric sweeps."""
        _check(lib.avs_dia_step_implicit(self.h, int(n), int(n_macro), int(n_micro)))

    def get_state(self):
        n = self.case.nleaves()
        vdf = np.zeros((3, self.case.nc, n))
        W = np.zeros((self.case.nc, self.case.dim + 3))
        _check(lib.avs_dia_get_state(self.h, vdf.ctypes.data, W.ctypes.data))
        return vdf, W

    def close(self):
        if getattr(self, "h", None):
            lib.avs_dia_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several Cases (same dimension, precision and non-default stream)
    advanced together by the batched kernels, optionally through a graph."""

    def __init__(self, cases):
        import torch
        self.cases = list(cases)
        n = len(self.cases)
        ptrs = (C.c_void_p * n)(*[c.ctx.value for c in self.cases])
        wb = lib.avs_batch_workspace_bytes(n)
        self.ws = torch.empty(max(wb, 1), dtype=torch.uint8, device=self.cases[0].device)
        b = C.c_void_p()
        _check(lib.avs_batch_create(n, ptrs, self.ws.data_ptr(), wb, C.byref(b)))
        self.b = b

    def step(self, n=1, graph=True):
        _check(lib.avs_batch_step(self.b, int(n), 1 if graph else 0))

    def check(self):
        _check(lib.avs_batch_check(self.b))

    def adapt(self, C1, C2):
        """Adapt every member (per-case thresholds); returns the new leaf counts."""
        n = len(self.cases)
        c1 = np.ascontiguousarray(np.broadcast_to(np.asarray(C1, np.float64), (n,)))
        c2 = np.ascontiguousarray(np.broadcast_to(np.asarray(C2, np.float64), (n,)))
        nn = np.zeros(n, np.int64)
        _check(lib.avs_batch_adapt(self.b, c1.ctypes.data, c2.ctypes.data, nn.ctypes.data))
        return nn

    def remap(self, correction=2):
        _check(lib.avs_batch_remap(self.b, int(correction)))

    def tune(self):
        """Tile choice by timing on the members' own state (left unchanged):
        pass-A leaf chunk per leaf-count bucket (<1024, <4096, <16384, more)
        and pass C's leaves in flight (1 or 2); returns the five choices."""
        ch = (C.c_int32 * 5)()
        _check(lib.avs_batch_tune(self.b, ch))
        return list(ch[:4]) + [int(ch[4]) + 1]

    def close(self):
        if getattr(self, "b", None):
            lib.avs_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
