"""Closed-form and independently integrated references used to pin the oracle.

Nothing here calls the oracle or the HIP library.  Each reference is derived
from the paper's physics (Sec. II and Sec. V) by a route that differs from the
oracle's discretisation: exact solutions, library ODE integrators, and a
generic covariant evaluation (Christoffel symbols from the metric by automatic
differentiation) of the shear tensor's projector definition.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import solve_ivp

from hydro_inputs.eos import C_SB, HBARC
from hydro_inputs.ics import Grid

# ---------------------------------------------------------------------------
# Bjorken flow (Sec. V.B)
# ---------------------------------------------------------------------------


def bjorken_ideal_exact(eps0, tau0, tau):
    """Ideal gas: eps = eps0 (tau0/tau)^(4/3)."""
    return eps0 * (tau0 / tau) ** (4.0 / 3.0)


def is_bjorken_rhs(etas):
    """0+1D Israel-Stewart Bjorken system, conformal EoS, y = (eps, Phi), Phi = -tau^2 pi^etaeta:
    d eps/d tau = -(eps + P - Phi)/tau,
    d Phi/d tau = -(Phi - 4 eta/(3 tau))/tau_pi - 4/3 Phi/tau,
    with eta = (eta/s)(eps+P) hbarc/T and tau_pi = 5 (eta/s) hbarc/T."""

    def f(tau, y):
        e, phi = y
        T = (e / C_SB) ** 0.25
        P = e / 3.0
        eta = etas * (e + P) * HBARC / T
        tpi = 5.0 * etas * HBARC / T
        return [-(e + P - phi) / tau, -(phi - 4.0 * eta / (3.0 * tau)) / tpi - 4.0 / 3.0 * phi / tau]

    return f


def bulk_bjorken_rhs(etas, zetas, taubulk_coef):
    """0+1D Bjorken system with shear, bulk pressure and a conserved density,
    conformal EoS, y = (eps, Phi, Pi, n):
    d eps/d tau = -(eps + P + Pi - Phi)/tau,
    d Phi/d tau = -(Phi - 4 eta/(3 tau))/tau_pi - 4/3 Phi/tau,
    d Pi/d tau = -(Pi + zeta/tau)/tau_Pi - 4/3 Pi/tau,
    d n/d tau = -n/tau (d_mu (n u^mu) = 0 with theta = 1/tau),
    eta = (eta/s) s hbarc, zeta = (zeta/s) s hbarc, s = (eps+P)/T, tau_pi = 5 (eta/s)
    hbarc/T, tau_Pi = taubulk_coef (zeta/s) hbarc/T."""

    def f(tau, y):
        e, phi, Pi, n = y
        T = (e / C_SB) ** 0.25
        P = e / 3.0
        s = (e + P) / T
        eta, zeta = etas * s * HBARC, zetas * s * HBARC
        tpi, tPi = 5.0 * etas * HBARC / T, taubulk_coef * zetas * HBARC / T
        return [-(e + P + Pi - phi) / tau,
                -(phi - 4.0 * eta / (3.0 * tau)) / tpi - 4.0 / 3.0 * phi / tau,
                -(Pi + zeta / tau) / tPi - 4.0 / 3.0 * Pi / tau,
                -n / tau]

    return f


def bulk_bjorken_reference(y0, tau0, tau1, etas, zetas, taubulk_coef):
    sol = solve_ivp(bulk_bjorken_rhs(etas, zetas, taubulk_coef), (tau0, tau1), list(y0),
                    method="DOP853", rtol=1e-13, atol=1e-16)
    return sol.y[:, -1]


def gubser_density(x, y, tau, L, n_hat0):
    """Conserved density on a Gubser flow of scale L: in the de Sitter frame
    d_rho (cosh^2 rho n^) = 0, so n^ = n_hat0 / cosh^2 rho and, with conformal weight
    3, n = n^ / tau^3, where (2 L tau cosh rho)^2 = L^4 + 2 L^2 (tau^2 + r^2) +
    (tau^2 - r^2)^2."""
    r2 = np.asarray(x, dtype=np.float64) ** 2 + np.asarray(y, dtype=np.float64) ** 2
    Q = L ** 4 + 2.0 * L * L * (tau * tau + r2) + (tau * tau - r2) ** 2
    cosh2 = Q / (2.0 * L * tau) ** 2
    return n_hat0 / cosh2 / tau ** 3


def is_bjorken_reference(eps0, phi0, tau0, tau1, etas):
    sol = solve_ivp(is_bjorken_rhs(etas), (tau0, tau1), [eps0, phi0], method="DOP853",
                    rtol=1e-13, atol=1e-16)
    return sol.y[0, -1], sol.y[1, -1]


def bjorken_ns_temperature(T0, tau0, tau, etas):
    """First-order (Navier-Stokes) Bjorken solution for the ideal gas:
    T/T0 = (tau0/tau)^(1/3) [1 + 2 (eta/s) hbarc/(3 T0 tau0) (1 - (tau0/tau)^(2/3))]."""
    r = tau0 / tau
    return T0 * r ** (1.0 / 3.0) * (1.0 + 2.0 * etas * HBARC / (3.0 * T0 * tau0) * (1.0 - r ** (2.0 / 3.0)))


# ---------------------------------------------------------------------------
# Riemann rarefaction (Sec. V.A)
# ---------------------------------------------------------------------------


def riemann_exact(zeta, cs):
    """Rarefaction into vacuum: eps/eps0 and v as functions of zeta = x/t."""
    zeta = np.asarray(zeta, dtype=np.float64)
    ratio = np.ones_like(zeta)
    fan = zeta >= -cs
    z = np.clip(zeta[fan], -cs, 1.0 - 1e-15)
    ratio[fan] = ((1.0 - cs) / (1.0 + cs) * (1.0 - z) / (1.0 + z)) ** ((1.0 + cs * cs) / (2.0 * cs))
    v = np.tanh(-cs / (1.0 + cs * cs) * np.log(np.maximum(ratio, 1e-300)))
    return ratio, v


# ---------------------------------------------------------------------------
# A uniformly moving fluid whose shear stress relaxes (exact IS solution).
# ---------------------------------------------------------------------------


def relaxing_fluid_milne(g: Grid, tau, eps0, v, a0, taupi):
    """Cartesian rest frame: u = gamma(1, v, 0, 0), pi_rest = diag(0, -a/2, -a/2, a) with
    a = a0 exp(-t'/tau_pi), t' = gamma (t - v x) the fluid's proper time.  This solves the
    Israel-Stewart equations exactly (sigma = theta = Du = 0 and d_mu pi^{mu nu} = 0).
    Returned in Milne tilde components on grid g at proper time tau."""
    X, _, E = g.mesh()
    gam = 1.0 / math.sqrt(1.0 - v * v)
    t = tau * np.cosh(E)
    tp = gam * (t - v * X)
    a = a0 * np.exp(-tp / taupi)
    L = np.array([[gam, gam * v, 0, 0], [gam * v, gam, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1.0]])
    shape = g.shape
    pic = np.zeros((4, 4) + shape)
    pr = np.zeros((4, 4) + shape)
    pr[1, 1] = -0.5 * a
    pr[2, 2] = -0.5 * a
    pr[3, 3] = a
    pic = np.einsum("ma,abxyz,nb->mnxyz", L, pr, L)
    ch, sh = np.cosh(E), np.sinh(E)
    # J^mu_alpha = d(tau, x, y, eta)/d(t, x, y, z); tilde scaling multiplies the eta row by tau
    Jt = np.zeros((4, 4) + shape)
    Jt[0, 0] = ch
    Jt[0, 3] = -sh
    Jt[1, 1] = 1.0
    Jt[2, 2] = 1.0
    Jt[3, 0] = -sh  # tau * (-sinh/tau)
    Jt[3, 3] = ch   # tau * (cosh/tau)
    pim = np.einsum("maxyz,abxyz,nbxyz->mnxyz", Jt, pic, Jt)
    order = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3)]
    pi = np.stack([pim[m, n] for m, n in order])
    ux = np.full(shape, gam * v)
    ue = -gam * sh
    return dict(eps=np.full(shape, eps0), ux=ux, uy=np.zeros(shape), ue=ue, pi=pi)


def conformal_taupi(eps0, etas):
    T = (eps0 / C_SB) ** 0.25
    return 5.0 * etas * HBARC / T


# ---------------------------------------------------------------------------
# Shear tensor from its projector definition, generic covariant derivatives.
# ---------------------------------------------------------------------------


def covariant_shear_milne(u_tilde_fn, X):
    """sigma~^{mu nu}, theta, and a~^nu = (D u)~^nu at Milne point X = (tau, x, y, eta).

    u_tilde_fn(X) -> (u~x, u~y, u~eta) as torch scalars.  The physical contravariant
    velocity is u = (u~^tau, u~x, u~y, u~eta / tau).  Christoffel symbols come from the
    metric g = diag(1, -1, -1, -tau^2) by automatic differentiation, and
    sigma^{mu nu} = 2 Delta^{mu nu alpha beta} nabla_alpha u_beta (Sec. II, eqn. projector).
    """
    import torch

    X = torch.tensor(X, dtype=torch.float64)

    def metric(Y):
        return torch.diag(torch.stack([torch.ones((), dtype=torch.float64),
                                       -torch.ones((), dtype=torch.float64),
                                       -torch.ones((), dtype=torch.float64), -Y[0] ** 2]))

    def ucontra(Y):
        ux, uy, ue = u_tilde_fn(Y)
        ut = torch.sqrt(1.0 + ux * ux + uy * uy + ue * ue)
        return torch.stack([ut, ux, uy, ue / Y[0]])

    g = metric(X)
    ginv = torch.linalg.inv(g)
    dg = torch.autograd.functional.jacobian(metric, X)  # dg[a, b, c] = d_c g_ab
    Gam = 0.5 * (torch.einsum("ad,dcb->abc", ginv, dg) + torch.einsum("ad,dbc->abc", ginv, dg)
                 - torch.einsum("ad,bcd->abc", ginv, dg))  # Gamma^a_{bc}
    u = ucontra(X)
    du = torch.autograd.functional.jacobian(ucontra, X)  # du[a, b] = d_b u^a
    nab = du.T + torch.einsum("abc,c->ba", Gam, u)  # nab[b, a] = nabla_b u^a
    theta = torch.trace(nab)
    Du = torch.einsum("b,ba->a", u, nab)
    Delta = ginv - torch.outer(u, u)
    nab_low = torch.einsum("ag,bg->ab", nab, g)  # nabla_alpha u_beta
    P4 = 0.5 * (torch.einsum("ma,nb->mnab", Delta, Delta) + torch.einsum("mb,na->mnab", Delta, Delta)) \
        - torch.einsum("mn,ab->mnab", Delta, Delta) / 3.0
    sig = 2.0 * torch.einsum("mnab,ab->mn", P4, nab_low)
    tau = X[0]
    scale = torch.tensor([1.0, 1.0, 1.0, float(tau)], dtype=torch.float64)
    sig_t = sig * scale[:, None] * scale[None, :]
    a_t = Du * scale
    order = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3)]
    return (np.array([float(sig_t[m, n]) for m, n in order]), float(theta),
            a_t.detach().numpy().copy())


# ---------------------------------------------------------------------------
# Viscous Gubser flow (Sec. V.C) mapped back by automatic differentiation.
# ---------------------------------------------------------------------------


def gubser_viscous_by_weyl(X, L, lambda1_hat, eps_hat0):
    """(eps, u~x, u~y, pi~[10]) at Milne point X = (tau, x, y, eta), x or y != 0.

    Evaluates the de Sitter-frame solution (eps^ = eps_hat0 cosh(rho)^(2/lambda1_hat - 8/3),
    u^ = (1, 0, 0, 0), pi^^{eta eta} = C = 2 eps^/lambda1_hat, pi^^{theta theta} cosh^2 rho =
    pi^^{phi phi} cosh^2 rho sin^2 theta = -C/2) and maps it back by the rules of Sec. V.C:
    eps = eps^/tau^4, u_mu = tau d rho/dx^mu, pi_{mu nu} = tau^-2 (dx^a/dx^mu)(dx^b/dx^nu) pi^_{ab},
    with the Jacobian of (rho, theta, phi, eta)(tau, x, y, eta) from automatic
    differentiation and indices raised with the Milne metric diag(1, -1, -1, -tau^2).
    """
    import torch

    X = torch.tensor(X, dtype=torch.float64)

    def hat(Y):
        tau, x, y, eta = Y[0], Y[1], Y[2], Y[3]
        r = torch.sqrt(x * x + y * y)
        rho = torch.asinh(-(L * L - tau * tau + r * r) / (2.0 * L * tau))
        th = torch.atan2(2.0 * L * r, L * L + tau * tau - r * r)
        phi = torch.atan2(y, x)
        return torch.stack([rho, th, phi, eta])

    xh = hat(X)
    J = torch.autograd.functional.jacobian(hat, X)  # J[a, m] = d xhat^a / d x^m
    rho, th = xh[0], xh[1]
    ch = torch.cosh(rho)
    eps_h = eps_hat0 * ch ** (2.0 / lambda1_hat - 8.0 / 3.0)
    C = 2.0 * eps_h / lambda1_hat
    A = -0.5 * C
    # lower-index hat components: g^_thth = -cosh^2, g^_phph = -cosh^2 sin^2 theta, g^_etaeta = -1
    pih_low = torch.zeros((4, 4), dtype=torch.float64)
    pih_low[1, 1] = A * ch ** 2            # (A / cosh^2) * cosh^4
    pih_low[2, 2] = A * ch ** 2 * torch.sin(th) ** 2
    pih_low[3, 3] = C
    tau = X[0]
    pi_low = torch.einsum("am,bn,ab->mn", J, J, pih_low) / tau ** 2
    ginv = torch.diag(torch.stack([torch.ones((), dtype=torch.float64),
                                   -torch.ones((), dtype=torch.float64),
                                   -torch.ones((), dtype=torch.float64), -1.0 / tau ** 2]))
    pi_up = ginv @ pi_low @ ginv
    u_low = tau * J[0]
    u_up = ginv @ u_low
    scale = torch.tensor([1.0, 1.0, 1.0, float(tau)], dtype=torch.float64)
    pit = pi_up * scale[:, None] * scale[None, :]
    order = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3)]
    return (float(eps_h / tau ** 4), float(u_up[1]), float(u_up[2]),
            np.array([float(pit[m, n]) for m, n in order]), u_up.detach().numpy().copy())


# ---------------------------------------------------------------------------
# Volumes cut from boxes and simplices by a plane or a linear function.
# ---------------------------------------------------------------------------


def cube_plane_hot_fraction(w):
    """Fraction of the unit 3-cube where the linear function with corner values
    w[4 b0 + 2 b1 + b2] is > 0, by inclusion-exclusion over the corners:
    vol{g0 + sum_i g_i x_i > 0} = sum_v (-1)^(3-|v|) max(0, g(v))^3 / (6 g1 g2 g3),
    valid for g1 g2 g3 != 0 (the box-spline form of the cut volume).  The
    alternating sum cancels heavily, so it is evaluated with 60 significant
    digits (the corner values themselves are taken as exact)."""
    import mpmath
    with mpmath.workdps(60):
        wm = [mpmath.mpf(float(x)) for x in w]
        g0 = wm[0]
        g = (wm[4] - wm[0], wm[2] - wm[0], wm[1] - wm[0])
        assert all(x != 0 for x in g)
        s = mpmath.mpf(0)
        for b in range(8):
            v = ((b >> 2) & 1, (b >> 1) & 1, b & 1)
            val = g0 + sum(gi * vi for gi, vi in zip(g, v))
            s += (-1) ** (3 - sum(v)) * max(mpmath.mpf(0), val) ** 3
        return float(s / (6 * g[0] * g[1] * g[2]))


def tet_hot_fraction_dd(v):
    """Hot fraction of a tetrahedron with a linear function of vertex values v
    (pairwise distinct), as the divided difference of x_+^3:
    sum over v_i > 0 of v_i^3 / prod_{j != i} (v_i - v_j)."""
    s = 0.0
    for i, vi in enumerate(v):
        if vi > 0:
            den = 1.0
            for j, vj in enumerate(v):
                if j != i:
                    den *= vi - vj
            s += vi ** 3 / den
    return s


def cube_hot_fraction_dd(w):
    """Mean over the six Kuhn tetrahedra 000 -> +e_p -> +e_q -> 111 of the
    divided-difference hot fraction (w indexed 4 b0 + 2 b1 + b2)."""
    import itertools
    s = 0.0
    for perm in itertools.permutations(range(3)):
        b = 0
        v = [w[0]]
        for ax in perm:
            b |= 4 >> ax
            v.append(w[b])
        s += tet_hot_fraction_dd(v)
    return s / 6.0
