"""Pins of the exact Euler Riemann solver used for the fluid-limit check.

* The textbook Sod problem (gamma = 1.4; left (1, 0, 1), right
  (0.125, 0, 0.1)) has star pressure 0.30313 and star velocity 0.92745.
* Across the shock the Rankine-Hugoniot conditions hold (mass, momentum and
  energy fluxes in the shock frame); across the rarefaction fan the entropy
  p / rho^gamma and the Riemann invariant u + 2a/(gamma - 1) are constant;
  pressure and velocity are continuous across the contact.
"""
import math

import numpy as np
import pytest

from oracle import euler

SOD = ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1))


def test_textbook_sod_star_state():
    ps, us = euler.star_state(*SOD, 1.4)
    assert abs(ps - 0.30313) < 5e-6 and abs(us - 0.92745) < 5e-6


@pytest.mark.parametrize("gamma", [1.4, 2.0, 5.0 / 3.0])
def test_wave_relations(gamma):
    (rl, ul, pl), (rr, ur, pr) = SOD
    ps, us = euler.star_state(*SOD, gamma)
    # right shock: find its speed from the sampled jump, check Rankine-Hugoniot
    s = np.linspace(us + 1e-9, 4.0, 40001)
    rho, u, p = euler.sample(*SOD, gamma, s)
    k = int(np.argmax(rho < 0.5 * (rr + rho[0])))
    S = 0.5 * (s[k - 1] + s[k])
    r1, u1, p1 = rho[0], u[0], p[0]           # post-shock (star) state
    E = lambda r, uu, pp: pp / (gamma - 1.0) + 0.5 * r * uu * uu  # noqa: E731
    m0, m1 = rr * (ur - S), r1 * (u1 - S)
    assert abs(m0 - m1) < 1e-3 * abs(m0)
    assert abs((m0 * (ur - S) + pr) - (m1 * (u1 - S) + p1)) < 1e-3 * p1
    e0 = (E(rr, ur, pr) + pr) * ur - S * E(rr, ur, pr)
    e1 = (E(r1, u1, p1) + p1) * u1 - S * E(r1, u1, p1)
    assert abs(e0 - e1) < 1e-3 * abs(e1)
    # left rarefaction fan: entropy and the Riemann invariant
    al = math.sqrt(gamma * pl / rl)
    fan = np.linspace(-al + 1e-6, us - math.sqrt(gamma * ps / euler.sample(*SOD, gamma,
                                                                           np.array([us - 1e-9]))[0][0]) - 1e-6, 50)
    rf, uf, pf = euler.sample(*SOD, gamma, fan)
    np.testing.assert_allclose(pf / rf ** gamma, pl / rl ** gamma, rtol=1e-12)
    af = np.sqrt(gamma * pf / rf)
    np.testing.assert_allclose(uf + 2.0 * af / (gamma - 1.0), ul + 2.0 * al / (gamma - 1.0),
                               rtol=1e-12)
    # contact: p and u continuous, density jumps
    rc, uc, pc = euler.sample(*SOD, gamma, np.array([us - 1e-9, us + 1e-9]))
    assert abs(pc[0] - pc[1]) < 1e-12 and abs(uc[0] - uc[1]) < 1e-12 and rc[0] > rc[1]
