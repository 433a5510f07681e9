"""Linear stability of the three-dimensional (D3Q19) bulk step, two ways:

* measured on the reference (oracle/slbm3d.py): one step on a periodic
  12^3 box, linearised about the rest state, one Fourier mode at a time (the
  cos and sin perturbations of the 19 populations span a 38-dimensional
  invariant subspace; their responses give the real amplification matrix);
* written out here from the definitions in Fourier space, sharing nothing
  with the reference: streaming multiplies population i by exp(-i k.c_i),
  the collision (eq:coll) is linear about rest, with the equilibrium of
  eq:fieq (j including S/2, eq:moments), the source S = (mu - lambda) grad rho
  (eq:sourceterm) whose isotropic stencil has the symbol
  i 3 sum_i w_i c_i sin(k.c_i), and psi_i = 3 w_i c_i.S.

The two agree on the largest eigenvalue modulus at every sampled mode; the
analysis then shows, over a 24^3 grid of wave vectors, that the step is
neutral (|g| <= 1) at the configurations the 3-D workloads use (lambda = mu
with tau_bar 0.55, 0.6 and 0.7). Unlike two dimensions, the D3Q19 bulk is
still neutral at lambda/mu = 2 with tau_bar 0.55; it first grows between
lambda/mu = 2 and 2.25 and clearly at 2.5 (about 1.036 per step). Growth seen
at lambda/mu = 2 in three dimensions therefore comes from the boundary rules,
not from the bulk step.
"""
import math

import numpy as np
import pytest

from oracle.slbm3d import Oracle3D, equilibrium
from slbm_workloads import box3d as B

C = B.C3.astype(float)
W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
CS2 = 1 / 3
N = 12
EPS = 1e-7


def analytic(k, lam_over_mu, tau, mu_l=1 / 3):
    """Largest |eigenvalue| of the one-step map for wave vectors k ([3] or
    [K, 3]; lattice units: mu = 1/3, lambda = (lambda/mu)/3)."""
    k = np.atleast_2d(np.asarray(k, dtype=float))
    lam_l = lam_over_mu * mu_l
    Q = len(W)
    K = len(k)
    kc = k @ C.T                                                              # [K, Q]
    g = 1j * (1 / CS2) * np.einsum("q,qa,kq->ka", W, C, np.sin(kc))           # symbol of grad, [K, 3]
    # linear maps from the 19 populations to drho, j, P and S
    rho_row = np.ones(Q)
    S_rows = (mu_l - lam_l) * g[:, :, None] * rho_row[None, None, :]          # [K, 3, Q]
    j_rows = C.T[None] + 0.5 * S_rows                                         # [K, 3, Q]
    P_rows = np.einsum("ia,ib->abi", C, C)                                    # [3, 3, Q]
    Hc = np.einsum("ia,ib->iab", C, C) - CS2 * np.eye(3)[None]                # [Q, 3, 3]
    quad = np.einsum("abj,iab->ij", P_rows, Hc) - CS2 * np.trace(Hc, axis1=1, axis2=2)[:, None] * rho_row[None, :]
    feq = W[None, :, None] * (rho_row[None, None, :] + np.einsum("ia,kaj->kij", C, j_rows) / CS2
                              + quad[None] / (2 * CS2 * CS2))
    psi = W[None, :, None] * np.einsum("ia,kaj->kij", C, S_rows) / CS2
    eye = np.eye(Q)[None]
    coll = eye - (eye - feq) / tau + (1 - 1 / (2 * tau)) * psi
    M = np.exp(-1j * kc)[:, :, None] * coll
    out = np.abs(np.linalg.eigvals(M)).max(axis=1)
    return out[0] if K == 1 else out


def measured(a, lam_over_mu, tau):
    """Largest |eigenvalue| of the reference's one-step map on mode
    2 pi a / N (a an integer 3-vector)."""
    mu = 0.05
    box = B.periodic_box3(N, N, N, lam=lam_over_mu * mu, mu=mu, tau=tau)
    o = Oracle3D(box)
    f0 = np.broadcast_to(equilibrium(np.ones(1), np.zeros((3, 1)), np.zeros((3, 3, 1)))[:, 0][:, None, None, None],
                         (19, N, N, N)).copy()
    zz, yy, xx = np.mgrid[0:N, 0:N, 0:N]
    ph = 2 * math.pi * (a[0] * xx + a[1] * yy + a[2] * zz) / N
    cs, sn = np.cos(ph), np.sin(ph)
    nyq = (sn * sn).sum() < 1e-6 * (cs * cs).sum()
    A = np.zeros((38, 38))
    for col in range(19 if nyq else 38):
        jj, basis = col % 19, (cs if col < 19 else sn)
        f = f0.copy()
        f[jj] += EPS * basis
        o.set_populations(f)
        o.n = 0
        o.step(1)
        d = (o.populations() - f0) / EPS
        A[:19, col] = (d * cs).sum(axis=(1, 2, 3)) / (cs * cs).sum()
        if not nyq:
            A[19:, col] = (d * sn).sum(axis=(1, 2, 3)) / (sn * sn).sum()
    if nyq:
        A = A[:19, :19]
    return np.abs(np.linalg.eigvals(A)).max()


MODES = [(1, 0, 0), (2, 1, 0), (3, 3, 1), (5, 2, 4), (6, 0, 0), (4, 4, 4), (6, 6, 3), (1, 5, 2)]


@pytest.mark.parametrize("lam_over_mu,tau", [(1.0, 0.55), (2.0, 0.55), (0.5, 0.7)])
def test_reference_matches_the_fourier_analysis(lam_over_mu, tau):
    for a in MODES:
        k = 2 * math.pi * np.array(a, dtype=float) / N
        assert abs(measured(a, lam_over_mu, tau) - analytic(k, lam_over_mu, tau)) < 1e-6, a


def _grid_max(lam_over_mu, tau, n=24):
    ks = 2 * math.pi * np.arange(n) / n
    k = np.stack(np.meshgrid(ks, ks, ks, indexing="ij"), -1).reshape(-1, 3)[1:]
    return analytic(k, lam_over_mu, tau).max()


@pytest.mark.parametrize("lam_over_mu,tau", [(1.0, 0.55), (1.0, 0.6), (1.0, 0.7), (2.0, 0.55)])
def test_neutral_where_the_workloads_run(lam_over_mu, tau):
    assert _grid_max(lam_over_mu, tau) <= 1 + 1e-9


def test_grows_beyond_lambda_twice_mu():
    g = _grid_max(2.5, 0.55)
    assert 1.02 < g < 1.06
