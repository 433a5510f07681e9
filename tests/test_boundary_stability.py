"""Growth of small perturbations next to traction-free walls (section 4,
eq:abbcon with eq:bcchainneum): a 12 x 40 plate, periodic in x, with free
top and bottom walls, started from a random velocity field of amplitude
1e-6; the growth factor per step of max |j| over the second half of 3000
steps.

These pin the stability findings the workloads are built on: with the
paper's extrapolation of rho_bd and sigma_tt along the link (neumann_order
1) a surface mode grows by about 0.8 % per step at lambda = mu, tau_bar =
0.55 -- slow enough for the paper's runs of a few hundred steps, fatal over
thousands -- while taking them at the boundary site (order 0) is stable
there; above lambda = mu neither is (the paper shows lambda/mu <= 1 only).
"""
import numpy as np
import pytest

from oracle import Oracle
from slbm_workloads import geometry as G


def growth(lam_over_mu, tau, order, q=0.5, steps=3000):
    mu = 0.05
    n = 40
    p = G.build_plate(12, n, lam=lam_over_mu * mu, mu=mu, tau=tau,
                      walls=[G.HLine(-q, 0), G.HLine(n - 1 + q, 0)], groups=[G.BCGroup(G.NEUMANN, (0.0, 0.0))],
                      periodic_x=True, neumann_order=order)
    o = Oracle(p)
    rng = np.random.default_rng(0)
    o.init_fields(vel=1e-6 * rng.standard_normal((2, p.ny, p.nx)) * p.mask)
    o.step(steps // 2)
    a = np.abs(o.moments()[1]).max()
    o.step(steps // 2)
    b = np.abs(o.moments()[1]).max()
    return (b / a) ** (1.0 / (steps // 2))


@pytest.mark.parametrize("q", [0.5, 0.2])
def test_paper_rule_grows_on_free_walls_at_lambda_equal_mu(q):
    assert growth(1.0, 0.55, order=1, q=q) > 1.005


@pytest.mark.parametrize("q", [0.5, 0.2])
def test_boundary_site_values_are_stable_at_lambda_equal_mu(q):
    assert growth(1.0, 0.55, order=0, q=q) < 1.001


def test_both_rules_grow_at_lambda_twice_mu():
    assert growth(2.0, 0.6, order=0) > 1.02
    assert growth(2.0, 0.6, order=1) > 1.02
