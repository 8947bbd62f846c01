"""Host logic of the automatic velocity space (Sec. 3.5) in the library
against the oracle and the paper's printed tables.  CPU only: these entry
points compute on the host and launch nothing."""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import avs_params as AP



@pytest.fixture(scope="module")
def avs():
    import torch  # noqa: F401  (torch's HIP runtime first, as the GPU tests load it)
    from paper_2212_05645_amd import avs as mod
    return mod

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rows(name):
    return [l.split() for l in open(os.path.join(GOLDEN, name)) if l.strip() and not l.startswith("#")]


def close(a, b, tol=1e-14):
    return abs(a - b) <= tol * max(abs(a), abs(b), 1e-300)


FLOWS = [dict(dim=D, R=R, gamma=g, Ma=Ma, T_inf=Ti, T_wall=Tw * Ti, rdv_sigmas=k, direction=e)
         for D, R, g, Ma, Ti, Tw, k, e in itertools.product(
             (2, 3), (0.5, 1.0, 208.0), (5.0 / 3.0, 1.4), (0.0, 0.16, 2.0, 5.0, 5.45, 12.0, 30.0), (1.0, 273.0),
             (1.0, 3.99, 4.0, 10.0), (4.0, 7.0), ((1.0, 0.0, 0.0), (0.6, 0.8, 0.0)))
         if not (R == 208.0 and Ti == 1.0)]


@pytest.mark.parametrize("flow", FLOWS[::7] + FLOWS[3::11])
def test_library_matches_oracle(avs, flow):
    try:
        p, vs = avs.auto_params(**flow)
    except avs.AvsError as err:
        # a box finer than the solver's levels is refused; the oracle agrees on the level count
        o = AP.auto_params(AP.Flow(**flow))
        assert err.status == avs.AVS_E_INVALID and o['L_max'] - min(o['L_min'], o['L_max']) > 12
        return
    o = AP.auto_params(AP.Flow(**flow))
    for k in ('L_max', 'L_w', 'L_min', 'L_sep'):
        assert p[k] == o[k], k
    for k in ('T0', 'sigma_inf', 'sigma_0', 'sigma_w', 'U_inf', 'R_dv', 'h_min', 'C1', 'C2', 'k_sigma'):
        assert close(p[k], o[k]) or (math.isinf(p[k]) and math.isinf(o[k])), k
    assert all(abs(a - b) <= 1e-14 * max(1.0, abs(b)) for a, b in zip(p['centre'], o['centre']))
    ov = AP.vspace_of(o, flow['dim'])
    assert vs['base'] == tuple(ov['base']) and vs['max_level'] == ov['max_level']
    assert np.allclose(vs['lo'], ov['lo'], rtol=0, atol=1e-13) and np.allclose(vs['hi'], ov['hi'], rtol=0, atol=1e-13)
    assert vs['leaf_capacity'] == min(2 ** (flow['dim'] * o['L_max']), 2 ** 26)


@pytest.mark.parametrize("row", rows("cylinder_adaptive_test.txt"), ids=lambda r: f"Ma{r[0]}")
def test_library_cylinder_table(avs, row):
    p, vs = avs.auto_params(dim=2, R=0.5, gamma=5.0 / 3.0, Ma=float(row[0]), T_inf=1.0, T_wall=1.0)
    assert p['L_max'] == int(row[2])
    assert (vs['base'][0] << vs['max_level']) == 2 ** p['L_max']


@pytest.mark.parametrize("row", rows("sphere_rdv.txt"), ids=lambda r: f"Rdv{r[1]}")
def test_library_sphere_table(avs, row):
    p, _ = avs.auto_params(dim=3, R=0.5, gamma=1.4, Ma=float(row[0]), T_inf=1.0, T_wall=7.3,
                           rdv_sigmas=float(row[1]))
    assert round(p['h_min'], 3) == float(row[2])


def test_direction_is_normalised(avs):
    a, _ = avs.auto_params(dim=2, R=0.5, gamma=5.0 / 3.0, Ma=3.0, T_inf=1.0, T_wall=1.0, direction=(1.0, 0.0, 0.0))
    b, _ = avs.auto_params(dim=2, R=0.5, gamma=5.0 / 3.0, Ma=3.0, T_inf=1.0, T_wall=1.0, direction=(2.5, 0.0, 0.0))
    assert a == b


@pytest.mark.parametrize("bad", [dict(dim=4), dict(gamma=1.0), dict(R=0.0), dict(Ma=-1.0), dict(Ma=float("nan")),
                                 dict(T_inf=0.0), dict(T_wall=-1.0), dict(rho_inf=0.0), dict(rdv_sigmas=0.0),
                                 dict(h_std=0.0), dict(direction=(0.0, 0.0, 0.0)), dict(h_std=1e-9)])
def test_invalid_flow_is_refused(avs, bad):
    flow = dict(dim=2, R=0.5, gamma=5.0 / 3.0, Ma=3.0, T_inf=1.0, T_wall=1.0)
    flow.update(bad)
    with pytest.raises(avs.AvsError) as e:
        avs.auto_params(**flow)
    assert e.value.status == avs.AVS_E_INVALID
