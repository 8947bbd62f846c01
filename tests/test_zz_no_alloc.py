"""The entry point that allocates nothing (avs_moments_noalloc: its partial
sums live in the library's static device array) against avs_moments on the
same state: fields bit for bit, totals to rounding (another summation
order, relative 1e-13 of the largest total), on two calls in a row, the
second on a smaller case, and again after the first case has stepped."""
import numpy as np
import pytest

from workloads import fields as F
from workloads import meshes as MM

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def avs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_05645_amd import avs as mod
    return mod


def check_same(avs, cs):
    import torch
    f_ref, t_ref = cs.moments()
    out = torch.full_like(f_ref, float("nan"))
    f, t = cs.moments_noalloc(fields_out=out)
    assert torch.equal(f, f_ref)
    assert np.max(np.abs(t - t_ref)) <= 1e-13 * np.max(np.abs(t_ref))
    assert np.all(np.isfinite(t))
    return t


def test_noalloc_moments_match_avs_moments(avs):
    # large enough for several partial blocks (3 000 cells) with a ragged last block
    big = F.cylinder(nr=12, nth=250, box=8.0, base=8, max_level=1, r1=4.0, first=0.05)
    small_mesh = MM.box2d(5, 4, periodic=(True, True))
    small_prim = F.perturbed_uniform(small_mesh['ncells'], 2, 3, amp=0.1, uamp=0.3)
    vs = dict(dim=2, lo=(-6, -6), hi=(6, 6), base=(8, 8), max_level=1)
    gas = dict(R=1.0, Pr=2 / 3, omega=0.81, mu_ref=0.03, T_ref=1.0, model=1)
    a = avs.Case(big['mesh'], big['vspace'], big['gas'], big['dt'], big['venkat_K'], big['prim0'])
    b = avs.Case(small_mesh, vs, gas, 0.004, 1.0, small_prim)
    assert a.nc > 2 * 1024 and a.nc % 1024 != 0 and b.nc < 1024
    ta = check_same(avs, a)
    tb = check_same(avs, b)            # second call, smaller input: only its own partials are summed
    assert tb[0] < 0.1 * ta[0]
    a.step(2)
    check_same(avs, a)
    check_same(avs, b)
    # totals only, fields only
    _, t = a.moments_noalloc(fields_out=None, totals=True)
    _, t_ref = a.moments(fields=False)
    assert np.max(np.abs(t - t_ref)) <= 1e-13 * np.max(np.abs(t_ref))
    a.close()
    b.close()
