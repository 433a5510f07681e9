"""Mode-I stress intensity factor of the edge-crack plate from the stress
ahead of the tip, for the closed-form check against Freund's K^0.

The plate's top and bottom edges carry a step traction sigma0.  The two
dilatational waves reach the crack line together after t1 = (ny/2) / c_d
steps and superpose there to 2 sigma0, so the crack faces see a suddenly
applied opening load t* = 2 sigma0 at t1.  Ahead of the tip (at distance r,
averaging the two rows beside the crack line) the singular part of sigma_yy
gives K = (sigma_yy - 2 sigma0) sqrt(2 pi r).  The paper samples two cells
ahead of the tip; here r = 2.5 cells (the tip point lies half-way between two
columns).  K^2 = A^2 (t - t0) is fitted over a window, leaving the onset time
t0 free: the lattice rules respond to the step with a delay of some tens of
steps (the paper reports the same smoothing of the onset).
"""
import math

import numpy as np

import closed_forms as CF


def sif_series(step, sigma_yy, plate, sigma0, t1, lo=40, hi=100, r=2.5):
    """Advance with step(1) from t1 + lo - 5 to t1 + hi and fit K^2 = A^2 (t - t0).

    step(n) advances the solver; sigma_yy() returns the sigma_yy field [ny, nx].
    Returns (A / A_freund, t0 - t1)."""
    ymid = plate.ny // 2            # rows ymid - 1 and ymid border the crack line
    x = int(round(plate.crack_tip_x + r))
    ts, ks = [], []
    t = t1 + lo - 5
    step(t)
    while t <= t1 + hi:
        s = sigma_yy()
        syy = 0.5 * (s[ymid - 1, x] + s[ymid, x])
        if t >= t1 + lo:
            ts.append(t)
            ks.append((syy - 2 * sigma0) * math.sqrt(2 * math.pi * r))
        step(1)
        t += 1
    ts = np.array(ts, float)
    ks = np.array(ks)
    slope, icpt = np.polyfit(ts, ks ** 2, 1)
    A = math.sqrt(slope)
    nu = CF.nu_from_speed_ratio((plate.lam + 2 * plate.mu) / plate.mu)
    cd_cells_per_step = math.sqrt((plate.lam + 2 * plate.mu) / plate.mu / 3.0)
    A0 = CF.freund_k0(2 * sigma0, nu, cd_cells_per_step, 1.0)
    return A / A0, -icpt / slope - t1


def paper_crack_k1_window(step, sigma_xx, plate, lc=100.0, t_face=0.009615, every=2):
    """The paper's centred crack (section 5.2) past the first scattered
    waves.  Advances with step(every) to 2.1 l_c/c_d, sampling
    K = sigma_xx sqrt(2 pi r) at P_1, two cells ahead of the upper tip on the
    crack line (the mean of the four sites around that point).

    step(n) advances the solver; sigma_xx() returns the sigma_xx field
    [ny, nx] in user units.  Returns (tau, K, drift, t_steep, t_rayleigh):
    the sample times in units of l_c/c_d, the series, the largest relative
    change over [1, 1.75] l_c/c_d of K/K^1 against its value at l_c/c_d, the
    time of the steepest rise of K over [1.5, 2.1] l_c/c_d, and the arrival
    time of the Rayleigh waves from the other tip, l_c/c_R."""
    cd = math.sqrt((plate.lam + 2 * plate.mu) / plate.rho)
    cs = math.sqrt(plate.mu / plate.rho)
    dt = math.sqrt(plate.rho / (3.0 * plate.mu))
    nu = CF.nu_from_speed_ratio(cd * cd / (cs * cs))
    ts = t_face * plate.mu
    yc = (plate.ny - 1) / 2.0 + lc / 2.0 + 2.0      # P_1 in site coordinates
    xc = (plate.nx - 1) / 2.0
    rows = slice(int(math.floor(yc)), int(math.floor(yc)) + 2)
    cols = slice(int(math.floor(xc)), int(math.floor(xc)) + 2)
    n_end = int(2.1 * lc / cd / dt)
    T, K = [], []
    for n in range(0, n_end + 1, every):
        if n:
            step(every)
        T.append(n * dt)
        K.append(sigma_xx()[rows, cols].mean() * math.sqrt(2 * math.pi * 2.0))
    T, K = np.array(T), np.array(K)
    tau = T * cd / lc
    sel = (tau >= 1.0) & (tau <= 1.75)
    r = K[sel] / CF.freund_k1_curve(ts, nu, cd, cs, lc, T[sel])
    drift = float(np.abs(r / r[0] - 1).max())
    late = (tau >= 1.5) & (tau <= 2.1)
    t_steep = float(tau[late][np.argmax(np.gradient(K, T)[late])])
    return tau, K, drift, t_steep, cd / CF.rayleigh_speed(cs, cd)
