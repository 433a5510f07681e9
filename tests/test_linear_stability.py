"""Linear stability of the bulk step (section 3, eq:coll with eq:sourceterm),
measured on the CPU reference itself: one step on a periodic lattice,
linearised about the rest state, one Fourier mode at a time.  For wave vector
k the cos and sin perturbations of each of the nine populations span an
18-dimensional invariant subspace; their responses give the amplification
matrix, whose largest eigenvalue modulus is the growth factor per step.

The pinned values come from an independent von Neumann analysis of the same
scheme on a 97^2 grid of wave vectors: neutral (|g| = 1) for lambda/mu up to
1.7 at tau_bar = 0.55, growing by about 2.9 % per step at lambda/mu = 2 (the
reason the workloads take tau_bar = 0.6 above lambda/mu = 1.5), and neutral
again at tau_bar = 0.6.  The unstable band is narrow and short-waved: on the
48^2 grid used here the largest growth at lambda/mu = 2 is about 1.6 %.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import Oracle, equilibrium
from slbm_workloads import geometry as G

N = 48          # lattice side: wave vectors 2 pi (a, b) / N
EPS = 1e-7


def max_growth(lam_over_mu, tau, ks):
    mu = 0.05
    p = G.periodic_box(N, N, lam=lam_over_mu * mu, mu=mu, tau=tau)
    o = Oracle(p)
    f0 = np.repeat(equilibrium(1.0, (0.0, 0.0), (0.0, 0.0, 0.0))[:, None, None], N, 1).repeat(N, 2)
    yy, xx = np.mgrid[0:N, 0:N]
    worst = 0.0
    for a, b in ks:
        ph = 2 * math.pi * (a * xx + b * yy) / N
        c, s = np.cos(ph), np.sin(ph)
        # on the Nyquist lines sin(k.x) vanishes (up to rounding): cos part only
        nyq = (s * s).sum() < 1e-6 * (c * c).sum()
        A = np.zeros((18, 18))
        for col in range(9 if nyq else 18):
            j, basis = col % 9, (c if col < 9 else s)
            f = f0.copy()
            f[j] += EPS * basis
            o.set_populations(f)
            o.step(1)
            d = (o.populations() - f0) / EPS
            # project each component back on cos and sin of the same mode
            A[:9, col] = (d * c).sum(axis=(1, 2)) / (c * c).sum()
            if not nyq:
                A[9:, col] = (d * s).sum(axis=(1, 2)) / (s * s).sum()
        if nyq:
            A = A[:9, :9]
        worst = max(worst, np.abs(np.linalg.eigvals(A)).max())
    return worst


# the scheme is symmetric under x <-> y and reflections: b <= a covers all modes
KS = [(a, b) for a in range(0, N // 2 + 1) for b in range(0, a + 1) if (a, b) != (0, 0)]


@pytest.fixture(scope="module", autouse=True)
def one_thread():
    n = O.set_threads(0)
    O.set_threads(1)
    yield
    O.set_threads(n)


@pytest.mark.parametrize("lam_over_mu,tau", [(1.0, 0.55), (0.769, 0.55), (1.5, 0.55), (2.0, 0.6)])
def test_neutral(lam_over_mu, tau):
    assert max_growth(lam_over_mu, tau, KS) <= 1 + 1e-6


def test_unstable_at_lambda_twice_mu_with_tau_055():
    g = max_growth(2.0, 0.55, KS)
    assert 1.01 < g < 1.0286 + 1e-3, g
