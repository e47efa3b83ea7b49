"""Exact solution of the 1D Riemann problem for an ideal gas (Toro, "Riemann
Solvers and Numerical Methods for Fluid Dynamics", ch. 4: pressure function,
Newton iteration for p*, wave-pattern sampling).  Written for the tests; it is
pinned against Toro's tabulated star values of the Sod problem."""
import math

import numpy as np


def star_state(rl, ul, pl, rr, ur, pr, g=1.4):
    al, ar = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)

    def fk(p, rk, pk, ak):
        if p > pk:
            A = 2.0 / ((g + 1.0) * rk)
            B = (g - 1.0) / (g + 1.0) * pk
            s = math.sqrt(A / (p + B))
            return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (B + p))
        q = p / pk
        return (2.0 * ak / (g - 1.0) * (q ** ((g - 1.0) / (2.0 * g)) - 1.0),
                1.0 / (rk * ak) * q ** (-(g + 1.0) / (2.0 * g)))

    p = max(1e-10, 0.5 * (pl + pr))
    for _ in range(200):
        f1, d1 = fk(p, rl, pl, al)
        f2, d2 = fk(p, rr, pr, ar)
        dp = (f1 + f2 + ur - ul) / (d1 + d2)
        pn = max(1e-12, p - dp)
        if abs(pn - p) < 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    f1, _ = fk(p, rl, pl, al)
    f2, _ = fk(p, rr, pr, ar)
    u = 0.5 * (ul + ur) + 0.5 * (f2 - f1)
    return p, u


def sample(rl, ul, pl, rr, ur, pr, xi, g=1.4):
    """(rho, u, p) at the similarity coordinate xi = (x - x0)/t (array)."""
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    al, ar = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    gm1, gp1 = g - 1.0, g + 1.0
    xi = np.asarray(xi, dtype=float)
    rho, u, p = np.empty_like(xi), np.empty_like(xi), np.empty_like(xi)
    for n, s in np.ndenumerate(xi):
        if s <= us:
            if ps > pl:
                SL = ul - al * math.sqrt(gp1 / (2 * g) * ps / pl + gm1 / (2 * g))
                if s <= SL:
                    W = (rl, ul, pl)
                else:
                    W = (rl * (ps / pl + gm1 / gp1) / (gm1 / gp1 * ps / pl + 1.0), us, ps)
            else:
                SHL = ul - al
                asl = al * (ps / pl) ** (gm1 / (2 * g))
                STL = us - asl
                if s <= SHL:
                    W = (rl, ul, pl)
                elif s > STL:
                    W = (rl * (ps / pl) ** (1.0 / g), us, ps)
                else:
                    uu = 2.0 / gp1 * (al + gm1 / 2.0 * ul + s)
                    aa = 2.0 / gp1 * (al + gm1 / 2.0 * (ul - s))
                    W = (rl * (aa / al) ** (2.0 / gm1), uu, pl * (aa / al) ** (2.0 * g / gm1))
        else:
            if ps > pr:
                SR = ur + ar * math.sqrt(gp1 / (2 * g) * ps / pr + gm1 / (2 * g))
                if s >= SR:
                    W = (rr, ur, pr)
                else:
                    W = (rr * (ps / pr + gm1 / gp1) / (gm1 / gp1 * ps / pr + 1.0), us, ps)
            else:
                SHR = ur + ar
                asr = ar * (ps / pr) ** (gm1 / (2 * g))
                STR = us + asr
                if s >= SHR:
                    W = (rr, ur, pr)
                elif s <= STR:
                    W = (rr * (ps / pr) ** (1.0 / g), us, ps)
                else:
                    uu = 2.0 / gp1 * (-ar + gm1 / 2.0 * ur + s)
                    aa = 2.0 / gp1 * (ar - gm1 / 2.0 * (ur - s))
                    W = (rr * (aa / ar) ** (2.0 / gm1), uu, pr * (aa / ar) ** (2.0 * g / gm1))
        rho[n], u[n], p[n] = W
    return rho, u, p
