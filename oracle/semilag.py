"""Semi-Lagrangian Runge-Kutta (SL-RK2) building blocks (Section 3).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Characteristics (Section 3.1, the scheme of Mang et al. the paper adopts): with
a stationary velocity v,
    X*  = x - dt v(x),   v* = v o X*,   X = x - 1/2 dt (v* + v(x))
gives the departure point of the characteristic through node x one step back
in time; it serves equations integrated forward in time.  Equations integrated
backward in time use the mirrored scheme with +dt.  v o X* is the cubic spline
interpolant of v.

Transport along the characteristic (Section 3.1, RK along the characteristic;
Section 3.3 and Table 1 give each equation as D_t u = f): the RK scheme is
read as Heun's method (explicit trapezoid, second order).  For
D_t u = f(u) integrated from t_n to t_{n+1}:
    a  = P(u_n) o X,  b = P(f(u_n)) o X
    u* = a + dt b
    u_{n+1} = a + 1/2 dt (b + f(u*))
where P(.) o X is the cubic spline interpolant at the departure points.  The
backward-in-time equations -D_t u = f(u) step from t_{n+1} to t_n with the
mirrored departure points and the same formulas.
"""
from __future__ import annotations

import torch

from . import bspline
from .problem import velocity_grid_units


def characteristics(vgrid: torch.Tensor, dt: float, direction: int) -> torch.Tensor:
    """Departure-point displacements X - x in grid units, [d, *N].

    direction = -1: forward-in-time equations (X = x - 1/2 dt (v + v o (x - dt v)));
    direction = +1: backward-in-time equations (the mirrored scheme).
    """
    d = vgrid.shape[0]
    N = vgrid.shape[1:]
    vv = velocity_grid_units(vgrid, N)
    xs = bspline.grid_index(N) + direction * dt * vv
    vstar = torch.stack([bspline.evaluate(bspline.prefilter(vv[j], d), xs) for j in range(d)], 0)
    return direction * 0.5 * dt * (vv + vstar)


def interp_at(f: torch.Tensor, disp: torch.Tensor) -> torch.Tensor:
    """P(f) o X for a scalar grid field f [*N] or a stack of fields [c, *N]."""
    d = disp.shape[0]
    if f.ndim == d:
        return bspline.interp_samples(f, disp, d)
    return torch.stack([bspline.interp_samples(f[i], disp, d) for i in range(f.shape[0])], 0)


def heun_step(u_grid, f_of, disp, dt: float):
    """One Heun step along the characteristic for D_t u = f(u) on grid fields (no projection).

    u_grid: samples at the departure time; f_of: callable grid -> grid; disp:
    departure-point displacements.  Returns the samples at the arrival time.
    """
    a = interp_at(u_grid, disp)
    b = interp_at(f_of(u_grid), disp)
    ustar = a + dt * b
    return a + 0.5 * dt * (b + f_of(ustar))
