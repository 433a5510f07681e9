"""Growth of small disturbances next to traction-free walls (section 4,
eq:abbcon / eq:abbnoncon with eq:bcchainneum).

On the CPU reference: a 12 x 40 plate, periodic in x, free top and bottom
walls crossing the links at fraction q, started from a random velocity
field of amplitude 1e-6 and stepped as a power iteration (the disturbance is
scaled back to its starting size every 60 steps, so it stays in the linear
regime however fast it grows); the growth factor per step is the geometric
mean over the second half of the run.

Independently (tests/naive_wall_modes.py): the largest eigenvalue modulus of
the one-step map of the same strip, linearised about rest and built row by
row from the paper's equations, over the plate's wave numbers 2 pi m / 12.
The two must agree.

These pin the stability findings the workloads are built on: with the
paper's extrapolation of rho_bd and sigma_tt along the link (neumann_order
1) a surface mode grows by about 0.8 % per step at lambda = mu, tau_bar =
0.55 -- slow enough for the paper's runs of a few hundred steps, fatal over
thousands -- while taking them at the boundary site (order 0) is stable
there; above lambda = mu neither is (the paper shows lambda/mu <= 1 only).
"""
import numpy as np
import pytest

from naive_wall_modes import max_growth
from oracle import Oracle
from slbm_workloads import configs
from slbm_workloads import geometry as G

NX, NY = 12, 40


def growth(lam_over_mu, tau, order, q=0.5, steps=2400, every=60, amp=1e-6):
    mu = 0.05
    p = G.build_plate(NX, NY, lam=lam_over_mu * mu, mu=mu, tau=tau,
                      walls=[G.HLine(-q, 0), G.HLine(NY - 1 + q, 0)], groups=[G.BCGroup(G.NEUMANN, (0.0, 0.0))],
                      periodic_x=True, neumann_order=order)
    o = Oracle(p)
    rest = o.populations()
    rng = np.random.default_rng(0)
    o.init_fields(vel=amp * rng.standard_normal((2, p.ny, p.nx)) * p.mask)
    d = o.populations() - rest
    o.set_populations(rest + d * (amp / np.linalg.norm(d)))
    logs = []
    for _ in range(steps // every):
        o.step(every)
        d = o.populations() - rest
        a = np.linalg.norm(d)
        logs.append(np.log(a / amp) / every)
        o.set_populations(rest + d * (amp / a))
    return float(np.exp(np.mean(logs[len(logs) // 2:])))


CASES = [(lm, q, order) for lm in (1.0, 1.5, 2.0) for q in (0.5, 0.2) for order in (0, 1)]


@pytest.mark.parametrize("lam_over_mu,q,order", CASES)
def test_reference_growth_matches_the_independent_mode_analysis(lam_over_mu, q, order):
    tau = configs.tau_for(lam_over_mu)
    g_ref = growth(lam_over_mu, tau, order, q)
    g_eig = max_growth(NY, NX, lam_over_mu, tau, q, order)
    print(f"lambda/mu {lam_over_mu} q {q} order {order} tau {tau}: reference {g_ref:.5f}, modes {g_eig:.5f}")
    assert abs(g_ref - g_eig) < 2e-3, (g_ref, g_eig)


@pytest.mark.parametrize("q", [0.5, 0.2])
def test_paper_rule_grows_on_free_walls_at_lambda_equal_mu(q):
    assert growth(1.0, 0.55, order=1, q=q) > 1.005
    assert max_growth(NY, NX, 1.0, 0.55, q, 1) > 1.005


@pytest.mark.parametrize("q", [0.5, 0.2])
def test_boundary_site_values_are_stable_at_lambda_equal_mu(q):
    assert growth(1.0, 0.55, order=0, q=q) < 1.001
    assert max_growth(NY, NX, 1.0, 0.55, q, 0) < 1.001


def test_both_rules_grow_at_lambda_twice_mu():
    assert growth(2.0, 0.6, order=0) > 1.02
    assert growth(2.0, 0.6, order=1) > 1.02


def test_mode_analysis_is_neutral_without_walls_in_the_bulk_limit():
    """A check of the independent operator itself: on a strip whose walls
    reflect nothing (lambda = mu, where the source term vanishes, q = 1/2,
    boundary-site values) the rest state is a fixed point, and a uniform
    shift of density (k = 0) is neither amplified nor lost by one step: the
    map has the eigenvalue 1 with the rest-density eigenvector's moments."""
    from naive_wall_modes import step_operator
    H = 6
    A = step_operator(H, 0.0, 1.0 / 3.0, 1.0 / 3.0, 0.55, 0.5, 0)
    ev = np.linalg.eigvals(A)
    assert np.min(np.abs(ev - 1.0)) < 1e-10
