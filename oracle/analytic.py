"""Closed forms of the paper, and a finite-difference Fick reference, used to
pin the oracle and the GPU physics (test infrastructure only).

All in lattice units with c_s^2 = 1/3 and tau = 1 unless given.
"""
from __future__ import annotations

import math

import numpy as np

CS2 = 1.0 / 3.0


def psi_fn(kind: str):
    """psi and d psi/d rho for psi = rho or psi = 1 - exp(-rho) (Eq. (psifunc))."""
    if kind == "rho":
        return (lambda r: r), (lambda r: 1.0)
    return (lambda r: 1.0 - math.exp(-r)), (lambda r: math.exp(-r))


def diffusion_pair(ra: float, rb: float, g: float, kind: str, tau: float = 1.0):
    """D^{cc} and D^{c cbar} of Eq. (diffu-t-1) for c = A; Psi' read as d Psi/d rho."""
    p, dp = psi_fn(kind)
    rt = ra + rb
    d_aa = CS2 * (tau - 0.5) * rb / rt - CS2 * ra * p(rb) * g * dp(ra) / rt
    d_ab = -CS2 * (tau - 0.5) * ra / rt + CS2 * rb * p(ra) * g * dp(rb) / rt
    return d_aa, d_ab


def diffusion_small_gradient(ra: float, rb: float, g: float, kind: str, tau: float = 1.0) -> float:
    """D^c of the small-gradient limit (Sec. III A), grad rho^B = -grad rho^A."""
    p, dp = psi_fn(kind)
    rt = ra + rb
    return CS2 * (tau - 0.5) - CS2 / rt * (rb * p(ra) * g * dp(rb) + ra * p(rb) * g * dp(ra))


def film_rate_constant(D: float, rho_ma: float, rho_mi: float, rho_h: float) -> float:
    """K in the film law: d x_I/dt = -K/(x_H - x_I - d0), Eqs. (xit)/(xt) with
    the sign fixed so that x_I decreases when rho_mi > rho_H."""
    return D * (rho_mi - rho_h) / (rho_ma - rho_mi / 2 - rho_h / 2)


def film_interface(t: float, x0: float, x_h: float, d0: float, K: float) -> float:
    """x_I(t) = x_H - d0 - sqrt((x_H - d0 - x0)^2 + 2 K t), the solution of the
    sign-fixed Eq. (xit) with x_I(0) = x0."""
    return x_h - d0 - math.sqrt((x_h - d0 - x0) ** 2 + 2.0 * K * t)


def droplet_mass(R: float, RH: float, d0: float, rho_ma: float, rho_mi: float, rho_h: float) -> float:
    """Eq. (drop-mass-1): mass of A in the sphere of radius R_H, by quadrature."""
    def integrand(r):
        if r < R - d0:
            return rho_ma
        if r < R + d0:
            return rho_mi - (rho_mi - rho_ma) * (R + d0 - r) / (2 * d0) * (R - d0) / r
        return rho_h - (rho_h - rho_mi) * (RH - r) / (RH - R - d0) * (R + d0) / r
    n = 20000
    h = RH / n
    s = 0.0
    for k in range(n):
        r = (k + 0.5) * h
        s += 4 * math.pi * r * r * integrand(r)
    return s * h


def droplet_dMdR(R: float, RH: float, d0: float, rho_ma: float, rho_mi: float, rho_h: float) -> float:
    """Eq. (mass-df2) without the factor dR/dt."""
    return (2 * math.pi / 3) * (
        RH ** 2 * (-rho_h + rho_mi)
        + RH * (-2 * R * rho_h + 2 * R * rho_mi - 2 * d0 * rho_h + 2 * d0 * rho_mi)
        + 6 * R ** 2 * rho_ma - 6 * R ** 2 * rho_mi - 2 * d0 ** 2 * rho_ma + 2 * d0 ** 2 * rho_mi)


def droplet_dMdt(R: float, RH: float, d0: float, D: float, rho_mi: float, rho_h: float) -> float:
    """Eq. (mass-df1) with the sign fixed: mass leaves when rho_mi > rho_H."""
    return -4 * math.pi * D * (rho_mi - rho_h) * (R + d0) * RH / (RH - R - d0)


def droplet_rate_plain(R, RH, d0, D, rho_ma, rho_mi, rho_h):
    """dR/dt of Eq. (mass-dfsum-sim) (no surface tension), sign-fixed."""
    return droplet_dMdt(R, RH, d0, D, rho_mi, rho_h) / droplet_dMdR(R, RH, d0, rho_ma, rho_mi, rho_h)


def laplace_densities(R, R0, gamma, rho_ma0, rho_mi0):
    """Eqs. (rho_ma) and (rho_mi): phase densities shifted by Laplace pressure."""
    rho_ma = rho_ma0 - 2 * gamma / CS2 * (1 / R0 - 1 / R)
    return rho_ma, rho_mi0 * rho_ma / rho_ma0


def droplet_dMdR_laplace(R, RH, d0, R0, gamma, rho_ma0, rho_mi0, rho_h):
    """Eq. (drop-mass-df4) without dR/dt, reading the symbol d as d0."""
    rho_ma, rho_mi = laplace_densities(R, R0, gamma, rho_ma0, rho_mi0)
    drho = -2 * gamma / (CS2 * R * R)          # d rho_ma / dR
    return (2 * math.pi / 3) * (
        (-RH ** 2 - 2 * R * RH - 2 * RH * d0) * rho_h
        + (RH ** 2 + 2 * R * RH + 2 * RH * d0 - 6 * R ** 2 + 2 * d0 ** 2) * rho_mi
        + (R * RH ** 2 + d0 * RH ** 2 + R ** 2 * RH + 2 * R * RH * d0 + d0 ** 2 * RH - 2 * R ** 3 + 2 * R * d0 ** 2)
        * (drho * rho_mi0 / rho_ma0)
        + (6 * R ** 2 - 2 * d0 ** 2) * rho_ma
        + (2 * R ** 3 - 2 * R * d0 ** 2) * drho)


def droplet_rate_laplace(R, RH, d0, D, R0, gamma, rho_ma0, rho_mi0, rho_h):
    """dR/dt of Eq. (drop-r-df4), sign-fixed, with the Laplace-shifted rho_mi."""
    _, rho_mi = laplace_densities(R, R0, gamma, rho_ma0, rho_mi0)
    return droplet_dMdt(R, RH, d0, D, rho_mi, rho_h) / droplet_dMdR_laplace(R, RH, d0, R0, gamma, rho_ma0,
                                                                            rho_mi0, rho_h)


def rk4(rate, y0: float, t_end: float, dt: float):
    """Classical fourth-order Runge-Kutta for dy/dt = rate(y); returns (t, y) lists."""
    ts, ys = [0.0], [y0]
    t, y = 0.0, y0
    while t < t_end - 1e-12:
        h = min(dt, t_end - t)
        k1 = rate(y)
        k2 = rate(y + 0.5 * h * k1)
        k3 = rate(y + 0.5 * h * k2)
        k4 = rate(y + h * k3)
        y = y + h * (k1 + 2 * k2 + 2 * k3 + k4) / 6
        t += h
        ts.append(t)
        ys.append(y)
    return ts, ys


def fick_bath_fd(nz: int, rho_h: float, D: float, T: float, dt: float = 0.05):
    """Explicit finite-difference solution of Fick's second law (Eq. (fick2))
    on nz nodes for the diffusion test of Sec. III A: the last node held at
    rho_H, a zero-flux mirror half a node below node 0 (a half-way
    bounce-back wall), zero initial density, integrated to time T."""
    u = np.zeros(nz)
    u[-1] = rho_h
    for _ in range(int(round(T / dt))):
        lap = np.empty(nz - 1)
        lap[1:] = u[2:] - 2 * u[1:-1] + u[:-2]
        lap[0] = u[1] - u[0]
        u[:-1] += dt * D * lap
    return u


def coexistence_single(G, guess=(0.1, 2.0)):
    """Liquid-vapour coexistence of the single-component model with psi = 1 -
    exp(-rho): equal bulk pressure p = c_s^2 rho + c_s^2 G psi^2 / 2 and
    int (p0 - p) psi' / psi^2 d rho = 0 over [rho_v, rho_l]. Both follow from
    mechanical equilibrium of a planar interface when the neighbour sum of
    Eq. (sc) is expanded to third order on a lattice isotropic to fourth
    order: the force's gradient term, psi times the third derivative of psi,
    divided by psi is an exact derivative."""
    from scipy.integrate import quad
    from scipy.optimize import fsolve
    cs2 = 1.0 / 3.0

    def psi(r):
        return 1.0 - np.exp(-r)

    def p(r):
        return cs2 * r + cs2 * G / 2 * psi(r) ** 2

    def eqs(v):
        rv, rl = v
        p0 = p(rv)
        return [p(rl) - p0, quad(lambda r: (p0 - p(r)) * np.exp(-r) / psi(r) ** 2, rv, rl)[0]]
    return fsolve(eqs, guess)
