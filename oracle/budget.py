"""Kinetic-energy budget of Sec. 3 by centred finite differences (numpy, FP64).

TEST INFRASTRUCTURE ONLY: used by ``tests/`` to check the GPU library's
energy-budget pass.  Nothing in the GPU package imports it.

From the macroscopic fields of the lattice at one time (rho_A, rho_B and the
hydrodynamic velocity u, each [ny][nx], x periodic), the averages over the
trimmed domain D (rows [trim, ny - trim), all columns) of

  pb        <u . grad p_b>                 p_b = c_s^2 rho + (G c_s^2 / 4)(rho^2 - phi^2)   (Eq. 12)
  korteweg  <u . (div P^K)>                P^K = [-kappa phi lap(phi) - (kappa/2)|grad phi|^2] I
                                                 + kappa grad phi (x) grad phi,  kappa = c_s^4 G / 4   (Eq. 13)
  ktau      <u . (div K^(tau))>            K^(tau) = c_s^4 (rho_A rho_B / rho)(tau - 1/2)^2 h (x) h,
                                                 h = grad rho_A / rho_A - grad rho_B / rho_B   (Eq. 14)
  viscous   <u . div(eta grad u + eta grad u^T)>,  eta = mean(rho) c_s^2 (tau - 1/2)   (Eq. 17, 19)

which enter the balance of Eq. 17: dE_k/dt = -(pb + korteweg + ktau) + viscous - buoyancy, with the
momentum-flux split of Eq. 19 (Eq. 11 gives P = p_b I + P^K + K^(tau)).

Discretisation (the paper only says centred differences): first derivatives
d_x q = (q(x+1) - q(x-1)) / 2 and likewise in y; the Laplacian of Eq. 13 is
the five-point sum q(x+1) + q(x-1) + q(y+1) + q(y-1) - 4 q; the divergence
of a tensor T is (div T)_b = d_x T_xb + d_y T_yb with the tensor formed at
each site first.  The isotropic part of Eq. 13 is read as (kappa/2)|grad
phi|^2 (the printed |grad phi^2| is taken as a typesetting slip).  eta is
the constant mean-density viscosity; tau is the mean of tau_A and tau_B.
Every site of D needs fields two rows away, so trim >= 2.
"""
from __future__ import annotations

import numpy as np

CS2 = 1.0 / 3.0   # lattice sound speed squared (Sec. 2)


def _dx(q):
    """Centred difference in x, periodic: (q(x+1) - q(x-1)) / 2."""
    return 0.5 * (np.roll(q, -1, axis=1) - np.roll(q, 1, axis=1))


def _dy(q):
    """Centred difference in y, (q(y+1) - q(y-1)) / 2; NaN on the first and
    last rows, where it is undefined."""
    out = np.full_like(q, np.nan)
    out[1:-1] = 0.5 * (q[2:] - q[:-2])
    return out


def _lap(q):
    """Five-point Laplacian; NaN on the first and last rows."""
    out = np.full_like(q, np.nan)
    out[1:-1] = (np.roll(q, -1, axis=1)[1:-1] + np.roll(q, 1, axis=1)[1:-1] + q[2:] + q[:-2]) - 4.0 * q[1:-1]
    return out


def integrands(rhoA, rhoB, ux, uy, G, tau):
    """Per-site integrands of the four budget terms ([ny][nx] each; NaN on
    the two rows next to each wall) and the viscosity-free viscous integrand
    u . div(grad u + grad u^T)."""
    rhoA, rhoB, ux, uy = (np.asarray(a, dtype=np.float64) for a in (rhoA, rhoB, ux, uy))
    rho = rhoA + rhoB
    phi = rhoA - rhoB
    # Eq. 12: bulk pressure
    pb = CS2 * rho + G * CS2 / 4.0 * (rho * rho - phi * phi)
    t_pb = ux * _dx(pb) + uy * _dy(pb)
    # Eq. 13: Korteweg tensor
    kappa = CS2 * CS2 * G / 4.0
    gx, gy = _dx(phi), _dy(phi)
    iso = -kappa * phi * _lap(phi) - 0.5 * kappa * (gx * gx + gy * gy)
    pxx = iso + kappa * gx * gx
    pxy = kappa * gx * gy
    pyy = iso + kappa * gy * gy
    t_k = ux * (_dx(pxx) + _dy(pxy)) + uy * (_dx(pxy) + _dy(pyy))
    # Eq. 14: the tau-dependent tensor
    hx = _dx(rhoA) / rhoA - _dx(rhoB) / rhoB
    hy = _dy(rhoA) / rhoA - _dy(rhoB) / rhoB
    c = CS2 * CS2 * (rhoA * rhoB / rho) * ((tau - 0.5) * (tau - 0.5))
    kxx = c * hx * hx
    kxy = c * hx * hy
    kyy = c * hy * hy
    t_tau = ux * (_dx(kxx) + _dy(kxy)) + uy * (_dx(kxy) + _dy(kyy))
    # viscous stress without eta: grad u + grad u^T
    sxx = 2.0 * _dx(ux)
    syy = 2.0 * _dy(uy)
    sxy = _dx(uy) + _dy(ux)
    t_v = ux * (_dx(sxx) + _dy(sxy)) + uy * (_dx(sxy) + _dy(syy))
    return {"pb": t_pb, "korteweg": t_k, "ktau": t_tau, "V": t_v}


def budget_from_fields(rhoA, rhoB, ux, uy, G, tau, trim=10):
    """Averages over the trimmed domain D of the budget terms (module doc)."""
    if trim < 2:
        raise ValueError("the budget stencils reach two rows: trim must be >= 2")
    ny = np.shape(rhoA)[0]
    if ny <= 2 * trim:
        raise ValueError("trimmed domain is empty")
    it = integrands(rhoA, rhoB, ux, uy, G, tau)
    D = slice(trim, ny - trim)
    out = {k: float(np.mean(v[D])) for k, v in it.items()}
    rho_mean = float(np.mean(np.asarray(rhoA, dtype=np.float64) + np.asarray(rhoB, dtype=np.float64)))
    eta = rho_mean * CS2 * (tau - 0.5)
    out["eta"] = eta
    out["viscous"] = eta * out["V"]
    return out
