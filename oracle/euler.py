"""Euler equations of gas dynamics (oracle, test infrastructure).

Conserved Q = (rho, rho u, rho v, rho E), fluxes f, g of eq. eulerTerms and the
ideal-gas closure p = (gamma-1)(rho E - rho (u^2+v^2)/2) of eq. eqn.eos.
Arrays carry the 4 conserved variables on the last axis.
"""
from __future__ import annotations

import numpy as np


def primitives(Q, gamma):
    rho = Q[..., 0]
    u = Q[..., 1] / rho
    v = Q[..., 2] / rho
    p = (gamma - 1.0) * (Q[..., 3] - 0.5 * rho * (u * u + v * v))
    return rho, u, v, p


def flux_f(Q, gamma):
    rho, u, v, p = primitives(Q, gamma)
    return np.stack([rho * u, rho * u * u + p, rho * u * v, u * (Q[..., 3] + p)], axis=-1)


def flux_g(Q, gamma):
    rho, u, v, p = primitives(Q, gamma)
    return np.stack([rho * v, rho * u * v, rho * v * v + p, v * (Q[..., 3] + p)], axis=-1)


def sound_speed(Q, gamma):
    rho, u, v, p = primitives(Q, gamma)
    return np.sqrt(gamma * p / rho)


def max_signal(Q, gamma):
    """|v| + c, the largest eigenvalue magnitude of the Euler Jacobian."""
    rho, u, v, p = primitives(Q, gamma)
    return np.sqrt(u * u + v * v) + np.sqrt(gamma * p / rho)
