"""Named synthetic workloads (grid, physics parameters, seeded initial state).

These stand in for the paper's event-by-event inputs (Trento/AMPT initial
states and lattice EoS tables are not available): sizes, spacings and value
distributions follow the benchmark configurations of the hot path.  Nothing
here computes any part of the step.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import eos as E
from . import ics


@dataclass
class Workload:
    name: str
    params: dict                 # nx, ny, ne, dx, dy, de, tau0, h, etas, viscous, cartesian
    eos: object                  # "conformal" or an EosTable
    steps: int
    ic: dict = None              # primitive initial state, or
    T4: object = None            # conserved initial state (4, nx, ny, ne)
    note: str = ""

    @property
    def ncell(self):
        p = self.params
        return p["nx"] * p["ny"] * p["ne"]

    @property
    def grid(self):
        p = self.params
        return ics.Grid(p["nx"], p["ny"], p["ne"], p["dx"], p["dy"], p["de"])


def _params(nx, ny, ne, dx, dy, de, tau0, h, etas=0.0, viscous=False, cartesian=False):
    return dict(nx=nx, ny=ny, ne=ne, dx=dx, dy=dy, de=de, tau0=tau0, h=h, etas=etas,
                viscous=int(viscous), cartesian=int(cartesian))


def gubser_ideal_33(steps: int = 50) -> Workload:
    """Ideal conformal hydro on 33x33x17 (dx = dy = deta = 0.3), tau0 = 1 fm,
    h = 0.02 fm, initial state = ideal Gubser flow (q = 1/fm, peak T = 0.4 GeV)."""
    p = _params(33, 33, 17, 0.3, 0.3, 0.3, 1.0, 0.02)
    g = ics.Grid(33, 33, 17, 0.3, 0.3, 0.3)
    return Workload("gubser_ideal_33x33x17", p, "conformal", steps, ic=ics.gubser_ideal(g, 1.0))


def gubser_viscous(n=41, ne=5, dx=0.3, de=0.3, h=0.02, steps=50, L=2.0, etas=0.2,
                   lambda1_hat=-10.0) -> Workload:
    """Second-order viscous conformal hydro started from the Sec. V.C Gubser
    solution at tau0 = 1 fm (L = 2 fm, eta/s = 0.2, lambda1_hat = -10, tau_pi
    coefficient from the solution's condition), boost invariant on ne cells."""
    p = _params(n, n, ne, dx, dx, de, 1.0, h, etas=etas, viscous=True)
    p.update(taupi_coef=ics.gubser_viscous_taupi_coef(lambda1_hat), lambda1_hat=lambda1_hat)
    g = ics.Grid(n, n, ne, dx, dx, de)
    return Workload(f"gubser_viscous_{n}x{n}x{ne}", p, "conformal", steps,
                    ic=ics.gubser_viscous(g, 1.0, L=L, lambda1_hat=lambda1_hat))


def hotspots_viscous(nx=201, ny=201, ne=105, dx=0.16, dy=0.16, de=0.3, steps=200, seed=1,
                     etas=0.08) -> Workload:
    """Viscous hydro, eta/s = 0.08, tau0 = 0.6 fm, h = 0.01 fm, 200 Gaussian hotspots
    (sigma 0.5 fm, Gamma(1) weights) in a 6.5 fm Woods-Saxon disk times an eta_s
    plateau (|eta_s| < 2, Gaussian tails sigma 1.3), peak e = 55 GeV/fm^3, zero
    initial flow and shear stress, 1555-row synthetic crossover EoS."""
    p = _params(nx, ny, ne, dx, dy, de, 0.6, 0.01, etas=etas, viscous=True)
    g = ics.Grid(nx, ny, ne, dx, dy, de)
    return Workload(f"hotspots_viscous_{nx}x{ny}x{ne}", p, E.cached_synthetic_table(), steps,
                    ic=ics.hotspots(g, seed=seed))


def hotspots_bulk(nx=201, ny=201, ne=105, dx=0.16, dy=0.16, de=0.3, steps=200, seed=1,
                  etas=0.08, zetas=0.04, baryon=True, n_peak=0.3) -> Workload:
    """hotspots_viscous with bulk viscosity zeta/s = 0.04 (tau_Pi coefficient 5) and the
    net-baryon density transported: Pi starts at zero, n = n_peak (e / e_max)^(3/4) fm^-3
    (the shape of an entropy density; n_peak = 0.3 fm^-3 about twice nuclear density)."""
    p = _params(nx, ny, ne, dx, dy, de, 0.6, 0.01, etas=etas, viscous=True)
    p.update(zetas=zetas, taubulk_coef=5.0, baryon=int(baryon))
    g = ics.Grid(nx, ny, ne, dx, dy, de)
    ic = ics.hotspots(g, seed=seed)
    ic["Pi"] = np.zeros(g.shape)
    ic["nb"] = n_peak * (ic["eps"] / ic["eps"].max()) ** 0.75 if baryon else None
    return Workload(f"hotspots_bulk_{nx}x{ny}x{ne}", p, E.cached_synthetic_table(), steps, ic=ic,
                    note="bulk pressure and baryon density")


def hotspots_minijets(nx=201, ny=201, ne=105, dx=0.16, dy=0.16, de=0.3, steps=200, seed=2,
                      etas=0.08) -> Workload:
    """As hotspots_viscous plus 400 mini-jet partons (p_T ~ Exp(2 GeV)) deposited into
    T~^{tau mu}; the initial flow follows from the root solve."""
    p = _params(nx, ny, ne, dx, dy, de, 0.6, 0.01, etas=etas, viscous=True)
    g = ics.Grid(nx, ny, ne, dx, dy, de)
    return Workload(f"hotspots_minijets_{nx}x{ny}x{ne}", p, E.cached_synthetic_table(), steps,
                    T4=ics.hotspots_with_minijets(g, 0.6, seed))


def minijets_defects(nx=33, ny=31, ne=9, dx=0.3, dy=0.3, de=0.4, steps=4, seed=2, n_each=6,
                     kinds=("nan", "momentum", "negative")):
    """hotspots_minijets on a small grid with defective cells planted in T~^{tau mu}
    (seeded positions inside the fireball, n_each of each kind in `kinds`): NaN in
    one component ("nan"), a momentum twice the energy, |T~^{tau i}| > T~^{tau tau}
    ("momentum"), and a negative energy T~^{tau tau} < 0 ("negative").  Input data
    only: it exercises the root solve's guards and the diagnostics counters."""
    wl = hotspots_minijets(nx, ny, ne, dx, dy, de, steps=steps, seed=seed)
    T4 = wl.T4.copy()
    rng = np.random.default_rng(seed + 31)
    hot = np.argwhere(T4[0] > 0.5 * T4[0].max())
    pick = hot[rng.choice(len(hot), 3 * n_each, replace=False)]
    for n, (i, j, k) in enumerate(pick):
        kind = n // n_each
        if ("nan", "momentum", "negative")[kind] not in kinds:
            continue
        if kind == 0:
            T4[n % 4, i, j, k] = np.nan
        elif kind == 1:
            T4[1 + n % 3, i, j, k] = 2.0 * T4[0, i, j, k]
        else:
            T4[0, i, j, k] = -0.1 * T4[0, i, j, k]
    wl.T4 = T4
    wl.name = f"minijets_defects_{'_'.join(kinds)}_{nx}x{ny}x{ne}"
    wl.note = "NaN, M > E and negative-energy cells"
    return wl


def gubser_dense_viscous(nx=201, ny=201, ne=105, dx=0.16, dy=0.16, de=0.3, steps=200,
                         etas=0.08) -> Workload:
    """The benchmark grid and physics with a smooth ideal-Gubser profile (q = 1/fm,
    evaluated at tau = 0.6 fm) instead of hotspots: no cell is vacuum."""
    p = _params(nx, ny, ne, dx, dy, de, 0.6, 0.01, etas=etas, viscous=True)
    g = ics.Grid(nx, ny, ne, dx, dy, de)
    return Workload(f"gubser_dense_viscous_{nx}x{ny}x{ne}", p, E.cached_synthetic_table(), steps,
                    ic=ics.gubser_ideal(g, 0.6), note="ideal Gubser profile at tau0, no vacuum")


def large_event(nx=385, ny=385, ne=129, dx=0.08, dy=0.08, de=0.15, steps=1000, seed=2,
                etas=0.08, h=0.005) -> Workload:
    """Large single event: 385x385x129 cells, dx = dy = 0.08 fm, deta = 0.15, h = 0.005 fm
    (the step of the 201^3-class grid scaled with the spacing, keeping the CFL number),
    tau0 = 0.6 fm, eta/s = 0.08, hotspots + mini-jets initial state (seed 2)."""
    p = _params(nx, ny, ne, dx, dy, de, 0.6, h, etas=etas, viscous=True)
    g = ics.Grid(nx, ny, ne, dx, dy, de)
    return Workload(f"large_event_{nx}x{ny}x{ne}", p, E.cached_synthetic_table(), steps,
                    T4=ics.hotspots_with_minijets(g, 0.6, seed), note="hotspots + 400 mini-jets")


def event_batch(nev=64, seed0=1000, steps=200, sizes=None):
    """A batch of uneven viscous events: nx = ny drawn uniformly from the odd
    numbers 101..301, n_eta from {1 (boost invariant), 33, 65, 105}, eta/s from
    {0 (ideal), 0.08, 0.16}; hotspot initial state with seed seed0 + e; spacings,
    tau0 and h as in the 201x201x105 benchmark grid.  `sizes` optionally overrides
    the drawn (n, n_eta, eta/s) triples (for small test batches)."""
    import numpy as np
    rng = np.random.default_rng(seed0)
    out = []
    for e in range(nev):
        if sizes is not None:
            n, ne, etas = sizes[e]
        else:
            n = int(rng.choice(np.arange(101, 302, 2)))
            ne = int(rng.choice([1, 33, 65, 105]))
            etas = float(rng.choice([0.0, 0.08, 0.16]))
        wl = hotspots_viscous(nx=n, ny=n, ne=ne, steps=steps, seed=seed0 + e, etas=etas)
        if etas == 0.0:
            wl.params["viscous"] = 0
        wl.name = f"event{e}_{n}x{n}x{ne}_etas{etas}"
        out.append(wl)
    return out


C1_FULL = dict(nx=201, ny=201, ne=105)
