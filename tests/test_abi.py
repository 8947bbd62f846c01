"""The C-ABI library loads, exports every symbol of include/avs.h, and
validates arguments on the host (no device work, runs without a GPU)."""
import ctypes as C
import re
from pathlib import Path

import numpy as np
import pytest

ROOT = Path(__file__).resolve().parents[1]


@pytest.fixture(scope="module")
def avs():
    import torch  # noqa: F401  (share torch's HIP runtime when present)
    from paper_2212_05645_amd import avs as mod
    return mod


def header_functions():
    h = (ROOT / "include" / "avs.h").read_text()
    return sorted(set(re.findall(r"^\s*(?:[a-z_0-9]+\s+\*?|const char \*)(avs_[a-z_]+)\(", h, re.M)))


def test_library_exports_every_declared_symbol(avs):
    declared = header_functions()
    assert len(declared) >= 19
    assert sorted(avs.EXPORTS) == declared
    for name in declared:
        assert hasattr(avs.lib, name)


def test_mu_ref_matches_mean_free_path_definition(avs):
    # hard-sphere: lambda = 16 mu / (5 rho sqrt(2 pi R T)) = Kn
    mu = avs.mu_ref_from_kn(0.075, 0.5, 1.0, 1.0, 1.0, 1.0)
    assert abs(16 * mu / (5 * np.sqrt(2 * np.pi)) - 0.075) < 1e-15


def descriptors(avs, dim=2, base=8, lmax=2, cap=None, precision=0):
    from workloads import meshes
    mesh = meshes.box2d(4, 3, periodic=(True, True)) if dim == 2 else meshes.box3d(2, 2, 2)
    keep = []

    def p(name, dt):
        a = np.ascontiguousarray(mesh[name], dtype=dt)
        keep.append(a)
        return a.ctypes.data
    pm = avs.avs_pmesh(dim=dim, ncells=mesh["ncells"], nfaces=mesh["nfaces"], cell_vol=p("cell_vol", np.float64),
                       cell_ctr=p("cell_ctr", np.float64), face_lr=p("face_lr", np.int64),
                       face_area=p("face_area", np.float64), face_nrm=p("face_nrm", np.float64),
                       face_ctr=p("face_ctr", np.float64), face_shift=p("face_shift", np.float64), nbc=0,
                       bc_kind=None, bc_state=None)
    vs = avs.avs_vspace(dim=dim, max_level=lmax)
    for d in range(dim):
        vs.base[d], vs.lo[d], vs.hi[d] = base, -5.0, 5.0
    vs.leaf_capacity = cap if cap is not None else base ** dim * 4 ** lmax
    op = avs.avs_opts(precision=precision, dt=1e-3, venkat_K=1.0)
    return vs, pm, op, keep, mesh


@pytest.mark.parametrize("dim", [2, 3])
def test_buffer_sizes(avs, dim):
    vs, pm, op, keep, mesh = descriptors(avs, dim=dim)
    P = 2 if dim == 2 else 1
    cap = -(-vs.leaf_capacity // 64) * 64
    rows = 2 * mesh["ncells"] + mesh["nfaces"]        # current, next and one interface row per face
    assert avs.lib.avs_vdf_bytes(C.byref(vs), C.byref(pm), C.byref(op)) == rows * P * cap * 8
    op.precision = 1
    assert avs.lib.avs_vdf_bytes(C.byref(vs), C.byref(pm), C.byref(op)) == rows * P * cap * 4
    assert avs.lib.avs_workspace_bytes(C.byref(vs), C.byref(pm), C.byref(op)) > 0


def test_invalid_arguments_are_rejected_before_device_work(avs):
    vs, pm, op, keep, mesh = descriptors(avs)
    bad = [("dim", lambda: setattr(vs, "dim", 4)), ("dt", lambda: setattr(op, "dt", 0.0)),
           ("capacity", lambda: setattr(vs, "leaf_capacity", 3)), ("precision", lambda: setattr(op, "precision", 7))]
    for what, mutate in bad:
        vs2, pm2, op2, keep2, _ = descriptors(avs)
        vs, pm, op = vs2, pm2, op2
        mutate()
        assert avs.lib.avs_vdf_bytes(C.byref(vs), C.byref(pm), C.byref(op)) == 0, what
        assert avs.lib.avs_last_error().decode() != "", what
    # init with null regions fails with AVS_E_INVALID and leaves no context behind
    vs, pm, op, keep, mesh = descriptors(avs)
    gas = avs.avs_gas(R=1.0, Pr=2 / 3, omega=0.5, mu_ref=0.05, T_ref=1.0, model=1)
    prim = np.tile([1.0, 0.0, 0.0, 1.0], (mesh["ncells"], 1))
    out = C.c_void_p(123)
    st = avs.lib.avs_init_mesh(C.byref(vs), C.byref(pm), C.byref(gas), C.byref(op), prim.ctypes.data, None, 0, None, 0,
                               None, C.byref(out))
    assert st == avs.AVS_E_INVALID and not out.value


def test_null_context_calls_fail_cleanly(avs):
    assert avs.lib.avs_step(None, 1, None) == avs.AVS_E_INVALID
    assert avs.lib.avs_remap(None, 2) == avs.AVS_E_INVALID
    avs.lib.avs_destroy(None)


def _cpu_only():
    import torch
    if torch.cuda.is_available():
        pytest.skip("host-side checks of avs_init_mesh use host pointers: CPU only")


def _init(avs, mesh, prim, dim=2):
    """avs_init_mesh on host stand-ins for the device regions (never reached:
    every call here stops in the host checks, or at the first HIP call on a
    machine without a GPU)."""
    vs, pm, op, keep, _ = descriptors(avs, dim=dim)
    keep.append(mesh)

    def p(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a.ctypes.data
    pm = avs.avs_pmesh(dim=dim, ncells=len(mesh["cell_vol"]), nfaces=len(mesh["face_area"]),
                       cell_vol=p(mesh["cell_vol"], np.float64), cell_ctr=p(mesh["cell_ctr"], np.float64),
                       face_lr=p(mesh["face_lr"], np.int64), face_area=p(mesh["face_area"], np.float64),
                       face_nrm=p(mesh["face_nrm"], np.float64), face_ctr=p(mesh["face_ctr"], np.float64),
                       face_shift=p(mesh["face_shift"], np.float64), nbc=0, bc_kind=None, bc_state=None)
    nv = avs.lib.avs_vdf_bytes(C.byref(vs), C.byref(pm), C.byref(op))
    nw = avs.lib.avs_workspace_bytes(C.byref(vs), C.byref(pm), C.byref(op))
    assert nv > 0 and nw > 0
    gas = avs.avs_gas(R=1.0, Pr=2 / 3, omega=0.5, mu_ref=0.05, T_ref=1.0, model=1)
    out = C.c_void_p(123)
    # 256-byte aligned addresses that are never dereferenced by the host checks
    fake = 1 << 40
    st = avs.lib.avs_init_mesh(C.byref(vs), C.byref(pm), C.byref(gas), C.byref(op),
                               p(prim, np.float64), fake, nv, fake + ((nv + 255) // 256) * 256, nw, None,
                               C.byref(out))
    assert not out.value
    return st, avs.lib.avs_last_error().decode()


def test_mesh_is_checked_on_the_host_before_device_work(avs):
    """Malformed meshes and states are refused by the host checks of
    avs_init_mesh with a message that names the fault; a well-formed mesh
    gets through them and stops at the first HIP call (no GPU here).  Run
    under the sanitizers, this walks the slot tables, least-squares
    coefficients, colouring and locality order of the host code."""
    _cpu_only()
    from workloads import meshes
    good = {k: np.array(v, copy=True) for k, v in meshes.box2d(4, 3, periodic=(True, True)).items()
            if isinstance(v, np.ndarray)}
    prim = np.tile([1.0, 0.0, 0.0, 1.0], (len(good["cell_vol"]), 1))

    def case(mutate, pr=prim):
        m = {k: v.copy() for k, v in good.items()}
        mutate(m)
        return _init(avs, m, pr)
    st, msg = case(lambda m: m["face_lr"].__setitem__((0, 0), 99))
    assert st == avs.AVS_E_INVALID and "L out of range" in msg
    st, msg = case(lambda m: m["face_lr"].__setitem__((1, 1), -5))
    assert st == avs.AVS_E_INVALID and "R out of range" in msg
    st, msg = case(lambda m: m["face_area"].__setitem__(2, -1.0))
    assert st == avs.AVS_E_INVALID and "negative area" in msg
    st, msg = case(lambda m: m["cell_vol"].__setitem__(3, 0.0))
    assert st == avs.AVS_E_INVALID and "non-positive volume" in msg
    # a fifth face on cell 0 (a duplicate of its first)
    def extra_face(m):
        for k in ("face_lr", "face_area", "face_nrm", "face_ctr", "face_shift"):
            m[k] = np.concatenate([m[k], m[k][:1]])
        f = int(np.nonzero((m["face_lr"] == 0).any(1))[0][0])
        m["face_lr"][-1] = m["face_lr"][f]
    st, msg = case(extra_face)
    assert st == avs.AVS_E_INVALID and "more than 4 faces" in msg
    bad = prim.copy()
    bad[5, 3] = -1.0
    st, msg = case(lambda m: None, bad)
    assert st == avs.AVS_E_INVALID and "not physical" in msg
    st, msg = case(lambda m: None)
    assert st == avs.AVS_E_HIP and "hipGetDevice" in msg


def test_separated_zone_arguments(avs):
    assert avs.lib.avs_set_separated(None, 1.0, 2.0, 1) == avs.AVS_E_INVALID
    assert "null context" in avs.lib.avs_last_error().decode()
