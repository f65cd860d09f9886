"""Equation-of-state inputs: the tables both the CPU oracle and the HIP path are fed.

The paper offers five equations of state (Sec. III, the EoS list after the
initial-condition discussion): the ideal gas EOSI (P = eps/3) and four tabulated
ones (lattice-wb2014, s95p-pce, EOSQ, pure gauge).  The tabulated data are not
available here, so a synthetic table of the same kind stands in for them: a
uniform grid in energy density with a smooth speed of sound that dips to 0.14
in a crossover region, 1555 rows.  This module only *produces* tables; the
lookup (interpolation and extrapolation) is part of the method and is written
separately on each side.

Units: eps, P in GeV/fm^3, T in GeV.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy import integrate, special

HBARC = 0.1973269804  # GeV fm
#: Stefan-Boltzmann constant of an ideal QGP with g = 47.5 degrees of freedom,
#: eps = C_SB * T^4 with T in GeV and eps in GeV/fm^3.
C_SB = 47.5 * math.pi ** 2 / 30.0 / HBARC ** 3

# Synthetic crossover parameters: cs2 = 1/3 - A exp(-ln^2(eps/EC)/(2 W^2)).
CS2_MIN = 0.14
A_DIP = 1.0 / 3.0 - CS2_MIN
EC = 0.45
W = 1.0


@dataclass(frozen=True)
class EosTable:
    """Uniform-eps table: row i holds (eps0 + i*deps, P, T, cs2)."""

    eps0: float
    deps: float
    P: np.ndarray
    T: np.ndarray
    cs2: np.ndarray

    @property
    def n(self) -> int:
        return int(self.P.shape[0])

    @property
    def eps(self) -> np.ndarray:
        return self.eps0 + self.deps * np.arange(self.n, dtype=np.float64)


def cs2_closed(eps):
    """Speed of sound squared of the synthetic crossover EoS (cs2(0) = 1/3)."""
    eps = np.asarray(eps, dtype=np.float64)
    out = np.full(eps.shape, 1.0 / 3.0)
    pos = eps > 0
    le = np.log(eps[pos] / EC)
    out[pos] = 1.0 / 3.0 - A_DIP * np.exp(-le * le / (2.0 * W * W))
    return out


def pressure_closed(eps):
    """P(eps) = int_0^eps cs2 de', in closed form via erf (x = ln(e'/EC))."""
    eps = np.asarray(eps, dtype=np.float64)
    out = np.zeros(eps.shape)
    pos = eps > 0
    X = np.log(eps[pos] / EC)
    dip = A_DIP * EC * math.exp(W * W / 2.0) * W * math.sqrt(math.pi / 2.0) * (
        1.0 + special.erf((X - W * W) / (W * math.sqrt(2.0))))
    out[pos] = eps[pos] / 3.0 - dip
    return out


def _cs2_scalar(e: float) -> float:
    if e <= 0.0:
        return 1.0 / 3.0
    le = math.log(e / EC)
    return 1.0 / 3.0 - A_DIP * math.exp(-le * le / (2.0 * W * W))


def _p_scalar(e: float) -> float:
    if e <= 0.0:
        return 0.0
    X = math.log(e / EC)
    return e / 3.0 - A_DIP * EC * math.exp(W * W / 2.0) * W * math.sqrt(math.pi / 2.0) * (
        1.0 + math.erf((X - W * W) / (W * math.sqrt(2.0))))


def _tail_integrand(x: float) -> float:
    # (3 cs2 - 1) / (4 (e + P)) de, with e = exp(x), de = e dx
    ep = math.exp(x)
    return (3.0 * _cs2_scalar(ep) - 1.0) / (4.0 * (ep + _p_scalar(ep))) * ep


def temperature_closed(eps):
    """T(eps) from dT/T = cs2 de/(e+P) at zero chemical potential.

    Normalised so the EoS approaches the Stefan-Boltzmann limit at large eps:
    ln T = 1/4 ln((e+P)/(4 C_SB/3)) - int_e^inf (3 cs2 - 1)/(4 (e'+P)) de'.
    The integrand is a narrow Gaussian bump in ln e, so the integral is done in
    x = ln e' and cut at 12 widths above the dip centre.
    """
    eps = np.atleast_1d(np.asarray(eps, dtype=np.float64))
    out = np.zeros(eps.shape)
    xmax = math.log(EC) + 12.0 * W
    order = np.argsort(-eps)
    acc, xprev = 0.0, xmax
    for idx in order:
        e = float(eps[idx])
        if e <= 0.0:
            continue
        x0 = math.log(e)
        if x0 < xprev:
            piece, _ = integrate.quad(_tail_integrand, x0, xprev, epsabs=1e-16, epsrel=1e-13,
                                      limit=200)
            acc += piece
            xprev = x0
        tail = acc if x0 < xmax else 0.0
        out[idx] = math.exp(0.25 * math.log((e + _p_scalar(e)) / (4.0 * C_SB / 3.0)) - tail)
    return out


def synthetic_table(n: int = 1555, deps: float = 0.04) -> EosTable:
    """The 1555-row synthetic crossover table (eps_i = 0.04 i GeV/fm^3)."""
    eps = deps * np.arange(n, dtype=np.float64)
    return EosTable(eps0=0.0, deps=deps, P=pressure_closed(eps), T=temperature_closed(eps),
                    cs2=cs2_closed(eps))


def conformal_temperature(eps):
    """T of the ideal-gas EoS (EOSI), eps = C_SB T^4."""
    return (np.asarray(eps, dtype=np.float64) / C_SB) ** 0.25


_CACHE: dict = {}


def cached_synthetic_table() -> EosTable:
    if "t" not in _CACHE:
        _CACHE["t"] = synthetic_table()
    return _CACHE["t"]
