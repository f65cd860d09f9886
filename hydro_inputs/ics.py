"""Seeded synthetic initial states for the hydro step.

Everything here is input generation only: coordinates, closed-form flow
profiles and random hotspot / parton placements.  None of the solver's
arithmetic (fluxes, sources, root solve, EoS lookup) lives here.  Both the CPU
oracle and the HIP library receive the arrays produced by these functions.

Conventions
-----------
Arrays have shape (nx, ny, ne) in C order (x slowest, eta_s fastest).  Cell
centres sit at x_i = (i - (nx-1)/2) dx, likewise for y and eta_s.  Velocities
are the tilde components u~ = (u^x, u^y, tau u^eta) of Sec. II; u~^tau follows
from normalisation.  pi~ components are ordered
(tautau, taux, tauy, taueta, xx, xy, xeta, yy, yeta, etaeta).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .eos import C_SB

PI_NAMES = ("tt", "tx", "ty", "te", "xx", "xy", "xe", "yy", "ye", "ee")


@dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    ne: int
    dx: float
    dy: float
    de: float

    @property
    def shape(self):
        return (self.nx, self.ny, self.ne)

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.ne

    def axes(self):
        x = (np.arange(self.nx) - (self.nx - 1) / 2.0) * self.dx
        y = (np.arange(self.ny) - (self.ny - 1) / 2.0) * self.dy
        e = (np.arange(self.ne) - (self.ne - 1) / 2.0) * self.de
        return x, y, e

    def mesh(self):
        x, y, e = self.axes()
        return np.meshgrid(x, y, e, indexing="ij")


def _zeros(g: Grid):
    return np.zeros(g.shape, dtype=np.float64)


def empty_pi(g: Grid) -> np.ndarray:
    return np.zeros((10,) + g.shape, dtype=np.float64)


# --------------------------------------------------------------------------
# Gubser flow (ideal limit), Sec. V.C: boost invariant, conformal EoS.
# --------------------------------------------------------------------------
def gubser_profile(x, y, tau, q=1.0, eps_peak_tau1=None, eps_hat=None):
    """Ideal Gubser flow at proper time tau (q = 1/L in fm^-1).

    eps = eps_hat (2q)^(8/3) / (tau^(4/3) [1 + 2 q^2 (tau^2 + r^2) + q^4 (tau^2 - r^2)^2]^(4/3)),
    v_r = 2 q^2 tau r / (1 + q^2 tau^2 + q^2 r^2)   (outward).
    ``eps_peak_tau1`` fixes eps_hat through eps(tau = 1/q, r = 0) = eps_hat q^(4/3).
    Returns (eps, u~x, u~y).
    """
    if eps_hat is None:
        eps_hat = eps_peak_tau1 / q ** (4.0 / 3.0)
    r2 = x * x + y * y
    den = 1.0 + 2.0 * q * q * (tau * tau + r2) + q ** 4 * (tau * tau - r2) ** 2
    eps = eps_hat * (2.0 * q) ** (8.0 / 3.0) / (tau ** (4.0 / 3.0) * den ** (4.0 / 3.0))
    a = 2.0 * q * q * tau / (1.0 + q * q * tau * tau + q * q * r2)  # v_r / r
    vx, vy = a * x, a * y
    ut = 1.0 / np.sqrt(1.0 - vx * vx - vy * vy)
    return eps, ut * vx, ut * vy


def gubser_ideal(g: Grid, tau: float, q: float = 1.0, T_peak: float = 0.4):
    """Gubser IC on grid g at proper time tau; peak T at tau = 1/q, r = 0 (conformal EoS)."""
    eps_peak = C_SB * T_peak ** 4
    X, Y, _ = g.mesh()
    eps, ux, uy = gubser_profile(X, Y, tau, q=q, eps_peak_tau1=eps_peak)
    return dict(eps=eps, ux=ux, uy=uy, ue=_zeros(g))


# --------------------------------------------------------------------------
# Gubser flow of second-order viscous hydrodynamics, Sec. V.C.
# --------------------------------------------------------------------------
def gubser_viscous_taupi_coef(lambda1_hat: float) -> float:
    """tau_pi coefficient b (tau_pi = b (eta/s) hbarc / T) that meets the solution's
    condition eta^ lambda1^2 = 3 tau_pi^ for the conformal gas: there
    eta^ = (4/3)(eta/s) hbarc c_SB^(1/4) and tau_pi^ = b (eta/s) hbarc c_SB^(1/4),
    so b = 4 lambda1_hat^2 / 9, whatever eta/s and c_SB are."""
    return 4.0 * lambda1_hat * lambda1_hat / 9.0


def gubser_viscous_profile(x, y, tau, L, lambda1_hat, eps_hat0):
    """Closed form at proper time tau (conformal EoS; L in fm).

    In the de Sitter frame the solution is eps^ = eps_hat0 cosh(rho)^-k with
    k = 8/3 - 2/lambda1_hat, u^ = (1, 0, 0, 0) and pi^^{eta eta} = C = (2/lambda1_hat) eps^,
    A = B = -C/2.  Mapped back (eps = eps^/tau^4, pi_{mu nu} = tau^-2 dx^/dx dx^/dx pi^),
    with Q = L^4 + 2 L^2 (tau^2 + r^2) + (tau^2 - r^2)^2 = (2 L tau cosh rho)^2:
      pi~^{tau tau} = 4 A r^2 / (tau^2 Q),  pi~^{tau i} = 2 A x_i (L^2 + tau^2 + r^2) / (tau^3 Q),
      pi~^{ij} = A delta_ij / tau^4 + 4 A x_i x_j / (tau^2 Q),  pi~^{eta eta} = -2 A / tau^4,
    the other components zero; the velocity is the ideal one,
    v_r = 2 tau r / (L^2 + tau^2 + r^2).  eps_hat0 carries units GeV fm.
    Returns (eps, u~x, u~y, pi10) in the pi~ order of this module."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    r2 = x * x + y * y
    Q = L ** 4 + 2.0 * L * L * (tau * tau + r2) + (tau * tau - r2) ** 2
    cosh_rho = np.sqrt(Q) / (2.0 * L * tau)
    k = 8.0 / 3.0 - 2.0 / lambda1_hat
    eps_hat = eps_hat0 * cosh_rho ** (-k)
    eps = eps_hat / tau ** 4
    A = -eps_hat / lambda1_hat  # A = -C/2, C = 2 eps^/lambda1_hat
    S = L * L + tau * tau + r2
    vx = 2.0 * tau * x / S
    vy = 2.0 * tau * y / S
    ut = 1.0 / np.sqrt(1.0 - vx * vx - vy * vy)
    pi = np.zeros((10,) + np.shape(eps), dtype=np.float64)
    pi[0] = 4.0 * A * r2 / (tau * tau * Q)
    pi[1] = 2.0 * A * x * S / (tau ** 3 * Q)
    pi[2] = 2.0 * A * y * S / (tau ** 3 * Q)
    pi[4] = A / tau ** 4 + 4.0 * A * x * x / (tau * tau * Q)
    pi[5] = 4.0 * A * x * y / (tau * tau * Q)
    pi[7] = A / tau ** 4 + 4.0 * A * y * y / (tau * tau * Q)
    pi[9] = -2.0 * A / tau ** 4
    return eps, ut * vx, ut * vy, pi


def gubser_viscous(g: Grid, tau: float, L: float = 2.0, lambda1_hat: float = -10.0,
                   T_peak: float = 0.4):
    """Viscous Gubser state on grid g at proper time tau, normalised so that the
    temperature at r = 0 is T_peak at tau = 1 fm (conformal EoS)."""
    X, Y, _ = g.mesh()
    e1, _, _, _ = gubser_viscous_profile(0.0, 0.0, 1.0, L, lambda1_hat, 1.0)
    eps_hat0 = C_SB * T_peak ** 4 / float(e1)
    eps, ux, uy, pi = gubser_viscous_profile(X, Y, tau, L, lambda1_hat, eps_hat0)
    return dict(eps=eps, ux=ux, uy=uy, ue=_zeros(g), pi=pi)


# --------------------------------------------------------------------------
# Bjorken flow, Sec. V.B: uniform in (x, y, eta_s), u~ = (1, 0, 0, 0).
# --------------------------------------------------------------------------
def bjorken(g: Grid, eps0: float, phi0: float = 0.0):
    """Uniform state; phi0 = -pi~^{etaeta} = 2 pi~^{xx} = 2 pi~^{yy} (traceless, transverse)."""
    pi = empty_pi(g)
    pi[4] = 0.5 * phi0
    pi[7] = 0.5 * phi0
    pi[9] = -phi0
    return dict(eps=np.full(g.shape, eps0), ux=_zeros(g), uy=_zeros(g), ue=_zeros(g), pi=pi)


# --------------------------------------------------------------------------
# Riemann problem, Sec. V.A (Cartesian coordinates, step in one direction).
# --------------------------------------------------------------------------
def riemann(nx: int, dx: float, eps0: float):
    """1D step along x: eps0 where x <= 0, vacuum where x > 0 (grid ny = ne = 1)."""
    g = Grid(nx, 1, 1, dx, 1.0, 1.0)
    X, _, _ = g.mesh()
    eps = np.where(X <= 0.0, eps0, 0.0)
    return g, dict(eps=eps, ux=_zeros(g), uy=_zeros(g), ue=_zeros(g))


# --------------------------------------------------------------------------
# Static relaxing fluid seen in Milne coordinates (exact solution built here).
# --------------------------------------------------------------------------
def static_milne(g: Grid, tau: float, eps0: float, amp):
    """A fluid at rest in Cartesian coordinates with pi^zz = a, pi^xx = pi^yy = -a/2.

    In Milne coordinates u~ = (cosh eta, 0, 0, -sinh eta) and
    pi~^tautau = a sinh^2, pi~^taueta = -a sinh cosh, pi~^etaeta = a cosh^2,
    pi~^xx = pi~^yy = -a/2.  ``amp`` is a(eta) on the grid's eta axis (the
    caller evaluates a at t = tau cosh eta).
    """
    _, _, E = g.mesh()
    a = np.broadcast_to(np.asarray(amp, dtype=np.float64)[None, None, :], g.shape)
    sh, ch = np.sinh(E), np.cosh(E)
    pi = empty_pi(g)
    pi[0] = a * sh * sh
    pi[3] = -a * sh * ch
    pi[9] = a * ch * ch
    pi[4] = -0.5 * a
    pi[7] = -0.5 * a
    return dict(eps=np.full(g.shape, eps0), ux=_zeros(g), uy=_zeros(g), ue=-sh, pi=pi)


# --------------------------------------------------------------------------
# Advected decaying shear mode (Cartesian, exact solution built here).
# --------------------------------------------------------------------------
def advected_pi(nx: int, dx: float, eps0: float, vx: float, amp: float, width: float,
                x0: float = 0.0):
    """Uniform eps and v_x; pi~^{y eta}(x) = amp exp(-(x-x0)^2/(2 width^2)).

    pi^{y eta} is transverse to u = gamma(1, v, 0, 0) and traceless, and it
    does not enter T^{tau mu} or the x-flux of T, so the fluid stays uniform.
    """
    g = Grid(nx, 1, 1, dx, 1.0, 1.0)
    X, _, _ = g.mesh()
    gam = 1.0 / math.sqrt(1.0 - vx * vx)
    pi = empty_pi(g)
    pi[8] = amp * np.exp(-(X - x0) ** 2 / (2.0 * width * width))
    return g, dict(eps=np.full(g.shape, eps0), ux=np.full(g.shape, gam * vx), uy=_zeros(g),
                   ue=_zeros(g), pi=pi)


# --------------------------------------------------------------------------
# Fluctuating heavy-ion-like initial state: Gaussian hotspots.
# --------------------------------------------------------------------------
def _woods_saxon_xy(rng, n, R=6.5, a=0.5):
    """n points in the plane with density proportional to 1/(1+exp((r-R)/a))."""
    out = []
    rmax = R + 10.0 * a
    while len(out) < n:
        r = rmax * np.sqrt(rng.random(4 * n))           # uniform in the disk of radius rmax
        acc = rng.random(4 * n) < 1.0 / (1.0 + np.exp((r - R) / a))
        phi = 2.0 * math.pi * rng.random(4 * n)
        for rr, pp in zip(r[acc], phi[acc]):
            out.append((rr * math.cos(pp), rr * math.sin(pp)))
            if len(out) == n:
                break
    return np.array(out)


def eta_envelope(e, eta_flat=2.0, sigma_eta=1.3):
    """Plateau |eta_s| < eta_flat with Gaussian tails (the form of Table I's H(eta_s))."""
    d = np.maximum(np.abs(e) - eta_flat, 0.0)
    return np.exp(-d * d / (2.0 * sigma_eta * sigma_eta))


def hotspots(g: Grid, seed: int, n_spots: int = 200, sigma: float = 0.5, R: float = 6.5,
             a_ws: float = 0.5, eta_flat: float = 2.0, sigma_eta: float = 1.3,
             eps_max: float = 55.0):
    """Sum of n_spots Gaussian hotspots (width sigma, Gamma(k=1) weights) placed by a
    2D Woods-Saxon disk, times an eta_s plateau envelope, scaled to max eps = eps_max.
    Zero initial flow, zero pi."""
    rng = np.random.default_rng(seed)
    xy = _woods_saxon_xy(rng, n_spots, R=R, a=a_ws)
    w = rng.gamma(1.0, 1.0, n_spots)
    x, y, e = g.axes()
    prof = np.zeros((g.nx, g.ny))
    for (cx, cy), wk in zip(xy, w):
        gx = np.exp(-(x - cx) ** 2 / (2.0 * sigma * sigma))
        gy = np.exp(-(y - cy) ** 2 / (2.0 * sigma * sigma))
        prof += wk * np.outer(gx, gy)
    H = eta_envelope(e, eta_flat, sigma_eta) if g.ne > 1 else np.ones(1)
    eps = prof[:, :, None] * H[None, None, :]
    eps *= eps_max / eps.max()
    return dict(eps=eps, ux=_zeros(g), uy=_zeros(g), ue=_zeros(g))


def minijet_deposit(g: Grid, seed: int, n_jets: int = 400, mean_pt: float = 2.0,
                    sigma_r: float = 0.5, sigma_eta: float = 0.5, R: float = 6.5,
                    a_ws: float = 0.5, eta_range: float = 2.0):
    """Energy-momentum of n_jets massless partons spread over the grid.

    Parton k: p_T ~ Exp(mean_pt), phi ~ U[0, 2pi), (x, y) from the Woods-Saxon
    disk, eta_k ~ U(-eta_range, eta_range), rapidity y = eta_k.  At a cell with
    space-time rapidity eta its tilde momentum is
    p_T (cosh(y - eta), cos phi, sin phi, sinh(y - eta)); it is spread with a
    Gaussian in (r, eta_s) normalised so that sum_cells dT~ dx dy deta = p~.
    Returns dT~^{tau mu} with shape (4, nx, ny, ne) in GeV/fm^2.
    """
    rng = np.random.default_rng(seed)
    xy = _woods_saxon_xy(rng, n_jets, R=R, a=a_ws)
    pt = rng.exponential(mean_pt, n_jets)
    phi = 2.0 * math.pi * rng.random(n_jets)
    etak = rng.uniform(-eta_range, eta_range, n_jets) if g.ne > 1 else np.zeros(n_jets)
    x, y, e = g.axes()
    vol = g.dx * g.dy * g.de
    # each parton's profile is separable, gx(x) gy(y) ge(eta): the deposits of all
    # partons are one contraction over the parton index, (x y) x partons times
    # partons x eta, for each component
    gx = np.exp(-(x[None, :] - xy[:, :1]) ** 2 / (2.0 * sigma_r ** 2))      # (n_jets, nx)
    gy = np.exp(-(y[None, :] - xy[:, 1:2]) ** 2 / (2.0 * sigma_r ** 2))     # (n_jets, ny)
    if g.ne > 1:
        ge = np.exp(-(e[None, :] - etak[:, None]) ** 2 / (2.0 * sigma_eta ** 2))  # (n_jets, ne)
    else:
        ge = np.ones((n_jets, 1))
    norm = gx.sum(axis=1) * gy.sum(axis=1) * ge.sum(axis=1) * vol
    w = np.where(norm > 0.0, pt / np.where(norm > 0.0, norm, 1.0), 0.0)
    dy_ = etak[:, None] - e[None, :]                                          # (n_jets, ne)
    B = np.stack([w[:, None] * ge * np.cosh(dy_), (w * np.cos(phi))[:, None] * ge,
                  (w * np.sin(phi))[:, None] * ge, w[:, None] * ge * np.sinh(dy_)])
    A = (gx[:, :, None] * gy[:, None, :]).reshape(n_jets, g.nx * g.ny)        # (n_jets, nx ny)
    out = np.empty((4,) + g.shape)
    for c in range(4):
        out[c] = (A.T @ B[c]).reshape(g.shape)
    return out


def hotspots_with_minijets(g: Grid, tau0: float, seed: int, **kw):
    """Conserved initial state T~^{tau mu} = tau0 (eps, 0, 0, 0) + parton deposits.

    For a fluid at rest T^{tau tau} = eps and T^{tau i} = 0, so no EoS is needed
    to build the conserved variables; the root solve recovers (eps, u~).
    """
    prim = hotspots(g, seed, **kw)
    dT = minijet_deposit(g, seed + 7919)
    T = dT.copy()
    T[0] += tau0 * prim["eps"]
    return T


# --------------------------------------------------------------------------
# Random cell states for root-solve tests.
# --------------------------------------------------------------------------
def random_states(n: int, seed: int, eps_lo: float = 1e-6, eps_hi: float = 1e3,
                  vmax: float = 0.9999):
    """eps log-uniform in [eps_lo, eps_hi]; velocity isotropic with |v| uniform in [0, vmax].
    Returns (eps, u~[n, 3])."""
    rng = np.random.default_rng(seed)
    eps = np.exp(rng.uniform(math.log(eps_lo), math.log(eps_hi), n))
    v = vmax * rng.random(n)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    gam = 1.0 / np.sqrt(1.0 - v * v)
    return eps, (gam * v)[:, None] * d
