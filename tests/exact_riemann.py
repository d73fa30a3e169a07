"""Exact solution of the 1-D Riemann problem between two stiffened gases.

Textbook construction (pressure function of the ideal-gas exact solver with the
pressure shifted by p_inf on each side; each side keeps its own gamma and
p_inf).  Used only by the tests as an independent truth for the oracle.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


class Side:
    def __init__(self, rho, u, p, gamma, pinf):
        self.rho, self.u, self.p, self.g, self.pinf = rho, u, p, gamma, pinf
        self.P = p + pinf
        self.c = math.sqrt(gamma * self.P / rho)

    def f(self, ps):
        """Velocity jump across the wave connecting this side to pressure ps."""
        g, P, rho, c = self.g, self.P, self.rho, self.c
        Ps = ps + self.pinf
        if Ps > P:   # shock
            A = 2.0 / ((g + 1.0) * rho)
            B = (g - 1.0) / (g + 1.0) * P
            return (Ps - P) * math.sqrt(A / (Ps + B))
        return 2.0 * c / (g - 1.0) * ((Ps / P) ** ((g - 1.0) / (2.0 * g)) - 1.0)

    def rho_star(self, ps):
        g, P = self.g, self.P
        Ps = ps + self.pinf
        if Ps > P:
            mu = (g - 1.0) / (g + 1.0)
            return self.rho * (Ps / P + mu) / (mu * Ps / P + 1.0)
        return self.rho * (Ps / P) ** (1.0 / g)


class ExactRiemann:
    def __init__(self, left: Side, right: Side):
        self.L, self.R = left, right
        du = right.u - left.u
        lo = -min(left.pinf, right.pinf) + 1e-9 * max(left.P, right.P)
        hi = 1e3 * max(left.P, right.P)
        fn = lambda p: left.f(p) + right.f(p) + du
        self.p_star = brentq(fn, lo, hi, xtol=1e-12, rtol=1e-15, maxiter=500)
        self.u_star = 0.5 * (left.u + right.u) + 0.5 * (right.f(self.p_star) - left.f(self.p_star))
        self.rho_star_L = left.rho_star(self.p_star)
        self.rho_star_R = right.rho_star(self.p_star)

    # wave speeds --------------------------------------------------------------
    def left_wave(self):
        L, ps = self.L, self.p_star
        Ps = ps + L.pinf
        g = L.g
        if Ps > L.P:
            S = L.u - L.c * math.sqrt((g + 1) / (2 * g) * Ps / L.P + (g - 1) / (2 * g))
            return ("shock", S, S)
        cs = L.c * (Ps / L.P) ** ((g - 1) / (2 * g))
        return ("rarefaction", L.u - L.c, self.u_star - cs)

    def right_wave(self):
        R, ps = self.R, self.p_star
        Ps = ps + R.pinf
        g = R.g
        if Ps > R.P:
            S = R.u + R.c * math.sqrt((g + 1) / (2 * g) * Ps / R.P + (g - 1) / (2 * g))
            return ("shock", S, S)
        cs = R.c * (Ps / R.P) ** ((g - 1) / (2 * g))
        return ("rarefaction", self.u_star + cs, R.u + R.c)

    def sample(self, s: float):
        """(rho, u, p, phase) at similarity coordinate s = (x - x0)/t."""
        if s <= self.u_star:
            L = self.L
            kind, head, tail = self.left_wave()
            if kind == "shock":
                if s < head:
                    return L.rho, L.u, L.p, 2
                return self.rho_star_L, self.u_star, self.p_star, 2
            if s <= head:
                return L.rho, L.u, L.p, 2
            if s >= tail:
                return self.rho_star_L, self.u_star, self.p_star, 2
            g = L.g
            c = 2.0 / (g + 1.0) * (L.c + 0.5 * (g - 1.0) * (L.u - s))
            u = 2.0 / (g + 1.0) * (L.c + 0.5 * (g - 1.0) * L.u + s)
            rho = L.rho * (c / L.c) ** (2.0 / (g - 1.0))
            P = L.P * (c / L.c) ** (2.0 * g / (g - 1.0))
            return rho, u, P - L.pinf, 2
        R = self.R
        kind, head, tail = self.right_wave()
        if kind == "shock":
            if s > head:
                return R.rho, R.u, R.p, 1
            return self.rho_star_R, self.u_star, self.p_star, 1
        if s >= tail:
            return R.rho, R.u, R.p, 1
        if s <= head:
            return self.rho_star_R, self.u_star, self.p_star, 1
        g = R.g
        c = 2.0 / (g + 1.0) * (R.c - 0.5 * (g - 1.0) * (R.u - s))
        u = 2.0 / (g + 1.0) * (-R.c + 0.5 * (g - 1.0) * R.u + s)
        rho = R.rho * (c / R.c) ** (2.0 / (g - 1.0))
        P = R.P * (c / R.c) ** (2.0 * g / (g - 1.0))
        return rho, u, P - R.pinf, 1

    def profile(self, x: np.ndarray, x0: float, t: float):
        out = np.array([self.sample((xi - x0) / t)[:3] for xi in x])
        return out[:, 0], out[:, 1], out[:, 2]
