"""Reference semi-implicit time step (TEST INFRASTRUCTURE ONLY: used by the
test suite; the product path never imports it).

One step of the predictor/corrector of Section "Semi-implicit integration
scheme", restricted to what this path computes: the inviscid acceleration is
the body force g alone (no pressure: the weakly compressible solver around the
viscous solve is not part of this path) and the density is frozen (no
continuity equation).  With u^n the velocity and mu^n the viscosity at r^n:

  1. B* = u^n + (dt/2) g on fluid rows;  A^n(dt/2) V* = B*;  u* = V* (fluid)
  2. r* = r^n + (dt/2) u^n (fluid);  mu* = mu(r*, u*)
  3. B = u^n + dt g on fluid rows;  A*(dt) V = B;  u^{n+1} = V (fluid)
  4. r^{n+1} = r^n + (dt/2)(u^n + u^{n+1}) (fluid);  mu^{n+1} = mu(r^{n+1}, u^{n+1})

Wall particles keep their position and velocity (the prescribed wall
velocity); their right-hand side is u_w for the dynamic model and 2 u_w for
the dummy model (the wall rows of eqs. implicit-system-dyn-full and
implicit-system-dummy-full), and they keep their viscosity.  Positions are
wrapped into the box on periodic axes.  The viscosity update is the
Papanastasiou law of `papanastasiou` (Section "Non-Newtonian viscosity");
mu = None keeps the viscosity constant (Newtonian).  Solves: the oracle's
robust BiCGSTAB (`solve`) with the Jacobi scaling.
"""
from __future__ import annotations

import numpy as np

from . import FLUID_TYPE, Operator, papanastasiou, solve


def _wrap(pos, lo, period):
    out = pos.copy()
    for a in range(3):
        if period[a] > 0.0:
            out[:, a] = lo[a] + np.mod(out[:, a] - lo[a], period[a])
    return out


def _rhs(u, ptype, g, dt, wall):
    f = ptype == FLUID_TYPE
    B = np.zeros_like(u)
    B[f] = u[f] + dt * np.asarray(g, dtype=np.float64)[None, :]
    B[~f] = u[~f] if wall == 0 else 2.0 * u[~f]
    return B


def step(w, pos, u, mu, dt, g, papa=None, tol=1e-12):
    """One step from (pos, u, mu) of workload `w` (mass, rho, ptype, period,
    lo, h, wall, avg taken from it).  papa = (tau0, m, mu0) or None.
    Returns (pos, u, mu, info), info holding the half-step state (pos_half,
    u_half, mu_half) and the two solve reports (rep_half, rep_full)."""
    f = w.ptype == FLUID_TYPE
    lo = np.zeros(3) if w.lo is None else np.asarray(w.lo, dtype=np.float64)

    def op(p, m_, dt_):
        return Operator(pos=p, mass=w.mass, rho=w.rho, mu=m_, ptype=w.ptype, period=w.period, h=w.h,
                        dt=dt_, wall=w.wall, avg=w.avg, jacobi=True, lo=lo)

    def visc(p, v):
        if papa is None:
            return mu.copy()
        m_, _ = papanastasiou(op(p, mu, dt), v, *papa)
        return m_

    Vh, rh, _ = solve(op(pos, mu, 0.5 * dt), _rhs(u, w.ptype, g, 0.5 * dt, w.wall), X0=u, tol=tol)
    uh = u.copy()
    uh[f] = Vh[f]
    ph = pos.copy()
    ph[f] = pos[f] + (0.5 * dt) * u[f]
    ph = _wrap(ph, lo, w.period)
    muh = visc(ph, uh)
    V, rf, _ = solve(op(ph, muh, dt), _rhs(u, w.ptype, g, dt, w.wall), X0=uh, tol=tol)
    un = u.copy()
    un[f] = V[f]
    pn = pos.copy()
    pn[f] = pos[f] + (0.5 * dt) * (u[f] + un[f])
    pn = _wrap(pn, lo, w.period)
    mun = visc(pn, un)
    return pn, un, mun, dict(pos_half=ph, u_half=uh, mu_half=muh, rep_half=rh, rep_full=rf)
