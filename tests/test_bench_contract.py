"""bench.py's command-line contract, checked without a GPU."""
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""



def test_roofline_uses_the_methods_algorithmic_bytes():
    """The roofline object of a form counts the method's bytes (2 reads and
    1 write of the VDF per step: pass C 2 rows, the sweep 3 rows per node),
    with this design's interface bytes beside them; fake timings."""
    import types
    import numpy as np
    sys.path.insert(0, str(ROOT))
    import bench
    nc, nf, nv = 1000, 2008, 500
    w = types.SimpleNamespace(nc=nc, nf=nf, cfg={'mesh': {'face_lr': np.array([[0, 1]] * 1992 + [[0, -1]] * 16)}})
    prof = {"passA": (10.0, 10), "face_eqflux": (2.0, 10), "macro": (0.1, 10), "target": (1.0, 10),
            "passC": (12.0, 10), "criterion": (0.5, 1)}
    r = {"prof": prof, "prof_leaves": nv}
    roof, kern = bench.roofline_of(w, r, "fp64", 5000.0)
    nodes = nc * nv
    assert roof["bound"] == "hbm" and roof["kernel"] == "passC"
    np.testing.assert_allclose(roof["frac"], 32 * nodes / 1.2e-3 / 8e12)
    np.testing.assert_allclose(roof["sweep"]["frac"], 48 * nodes / (1.0 + 0.2 + 0.01 + 0.1 + 1.2) * 1e3 / 8e12)
    assert roof["passC"]["design_bytes_per_node"] == 16 * (2 + nf / nc)
    roof32, _ = bench.roofline_of(w, {"prof": dict(prof, passA=(20.0, 10)), "prof_leaves": nv}, "fp32", 5000.0)
    assert roof32["bound"] == "alu" and roof32["kernel"] == "passA"
    assert roof32["sweep"]["algorithmic_bytes_per_node"] == 24
