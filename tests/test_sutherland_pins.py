"""Pins of the Sutherland viscosity option of the oracle (Eq. Sutherland,
Sec. 4.6).  CPU only."""
import os

import pytest

from oracle import avs_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def gas(law, C_s=0.0, mu_ref=1.0, T_ref=1.0, omega=0.74):
    return O.Gas(R=1.0, Pr=2.0 / 3.0, omega=omega, mu_ref=mu_ref, T_ref=T_ref, model=1, law=law, C_s=C_s)


def test_textbook_air_value():
    row = [l.split() for l in open(os.path.join(GOLDEN, "sutherland.txt")) if l.strip() and not l.startswith("#")][0]
    mu0, T0, S, T, mu = (float(x) for x in row)
    got = O.viscosity(T, gas(1, C_s=S, mu_ref=mu0, T_ref=T0))
    assert float(f"{got:.3e}") == mu


def test_reference_state_and_limits():
    g = gas(1, C_s=2.5, mu_ref=0.3, T_ref=1.7)
    assert abs(O.viscosity(1.7, g) - 0.3) < 1e-16
    # hot gas: mu ~ T^(1/2); cold gas: mu ~ T^(3/2)
    assert abs(O.viscosity(4e6, g) / O.viscosity(1e6, g) - 2.0) < 1e-5
    assert abs(O.viscosity(4e-6, g) / O.viscosity(1e-6, g) - 8.0) < 1e-5


@pytest.mark.parametrize("law", [0, 1])
def test_tau_is_viscosity_over_pressure(law):
    g = gas(law, C_s=1.3)
    for rho, T in ((1.0, 1.0), (0.3, 4.2), (2.5, 0.25)):
        assert abs(O.tau(rho, T, g) * rho * g.R * T - O.viscosity(T, g)) <= 1e-15 * O.viscosity(T, g)


def test_power_law_unchanged():
    g = gas(0, omega=0.81, mu_ref=0.2, T_ref=1.0)
    assert abs(O.viscosity(3.0, g) - 0.2 * 3.0 ** 0.81) < 1e-15
