"""HIP library vs CPU oracle, element by element, through the C ABI.

FP64 bar: every field within 1e-12 of the oracle, relative to the field's
scale (max |ref| over the tensor's components; max u~^tau for velocities).
"""
import os
import sys

import numpy as np
import pytest

from hydro_inputs import eos as E
from hydro_inputs import ics
from hydro_inputs import workloads as W

from . import gpu_common as G

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _both(wl, steps, tol=TOL, threads=None, **kw):
    _say(f"{wl.name} steps={steps} kw={kw}")
    g = G.run_gpu(wl, steps, **kw)
    gf = g.fields()
    o = G.run_oracle(wl, steps, threads=threads, **kw)
    of = o.fields()
    rel = G.assert_parity(gf, of, tol, wl.name)
    return g, o, rel


def test_gubser_ideal_33x33x17_full():
    """Ideal conformal Gubser flow, 33x33x17, 50 steps (the small benchmark case)."""
    wl = W.gubser_ideal_33()
    g, o, rel = _both(wl, 50)
    dg, do = g.diag(), o.diag()
    assert abs(dg["eps_max"] - do["eps_max"]) <= 1e-12 * do["eps_max"]
    assert abs(dg["sum_Ttt"] - do["sum_Ttt"]) <= 1e-12 * abs(do["sum_Ttt"])
    assert abs(dg["geo_src"] - do["geo_src"]) <= 1e-11 * abs(do["geo_src"])


def test_viscous_hotspots_ragged():
    """Viscous, table EoS, ragged grid spanning several workgroups, 20 steps."""
    wl = W.hotspots_viscous(nx=45, ny=39, ne=13, dx=0.35, dy=0.35, de=0.4, steps=20, seed=5)
    g, o, rel = _both(wl, 20)
    dg, do = g.diag(), o.diag()
    for k in ("solves", "clamps", "nonconv", "nans", "vacuum"):
        assert abs(dg[k] - do[k]) <= max(2, 1e-6 * do["solves"]), (k, dg[k], do[k])
    assert abs(dg["newton_mean"] - do["newton_mean"]) < 0.01


def test_lambda1_hotspots_ragged():
    """The second-order lambda_1 term (lambda1_hat = -10, tau_pi coefficient 7.5)
    on the viscous hotspot state with the table EoS, ragged grid, 20 steps: every
    pi~ component and the cells it feeds back into."""
    wl = W.hotspots_viscous(nx=37, ny=41, ne=11, dx=0.35, dy=0.35, de=0.4, steps=20, seed=6)
    g, o, rel = _both(wl, 20, taupi_coef=7.5, lambda1_hat=-10.0)
    # the term must matter here: same run without it differs well above the bar
    f0 = G.run_oracle(wl, 20, taupi_coef=7.5).fields()
    d = G.compare(f0, o.fields())
    assert max(d[f"pi{m}"] for m in range(10)) > 1e-4, d


def test_viscous_gubser_second_order():
    """The Sec. V.C viscous Gubser flow (lambda_1 term, tau_pi from the solution's
    condition, conformal EoS), 41x41x5, 50 steps against the oracle; the GPU result
    also stays within 2% of the closed form for r <= 2 fm (0.9% and 0.6% in e and
    pi~^{eta eta} on this grid; convergence itself is pinned on the CPU)."""
    wl = W.gubser_viscous(steps=50)
    g, o, rel = _both(wl, 50)
    gf = g.fields()
    ex = ics.gubser_viscous(wl.grid, 1.0 + 50 * wl.params["h"])
    X, Y, _ = wl.grid.mesh()
    m = (X ** 2 + Y ** 2) <= 4.0
    assert np.abs(gf["eps"] - ex["eps"])[m].max() < 0.02 * ex["eps"][m].max()
    assert np.abs(gf["pi9"] - ex["pi"][9])[m].max() < 0.02 * np.abs(ex["pi"][9][m]).max()


def test_ideal_table_boost_invariant():
    """Ideal hydro with the table EoS on a 2+1D grid (ne = 1), 30 steps."""
    wl = W.hotspots_viscous(nx=61, ny=53, ne=1, dx=0.25, dy=0.25, de=0.3, steps=30, seed=3)
    wl.params["viscous"] = 0
    wl.params["etas"] = 0.0
    _both(wl, 30)


def test_cartesian_riemann():
    """Cartesian mode, step into vacuum along x, 100 steps."""
    g, ic = ics.riemann(200, 0.1, 10.0)
    p = dict(nx=200, ny=1, ne=1, dx=0.1, dy=1.0, de=1.0, tau0=1.0, h=0.025, etas=0.0,
             viscous=0, cartesian=1)
    wl = W.Workload("riemann_200", p, "conformal", 100, ic=ic)
    _both(wl, 100)


def test_minijets_conserved_initial_state():
    """Conserved initial state (hotspots + mini-jet momentum), viscous, 10 steps.

    Dilute cells that partons push close to light speed make this state
    ill-conditioned: the oracle alone answers a 1e-15 relative input perturbation
    with ~1e-6 in u~ after 10 steps.  The bar is therefore 1e-12 on cells with
    e >= 1 GeV/fm^3 (where that response is ~1e-14), and elsewhere no more than
    10x the oracle's own response to the 1e-15 perturbation (floor 1e-12)."""
    wl = W.hotspots_minijets(nx=41, ny=41, ne=9, dx=0.35, dy=0.35, de=0.45, steps=10, seed=4)
    _say(f"{wl.name} steps=10 (conditioning-aware)")
    gf = G.run_gpu(wl, 10).fields()
    of, sens = G.conditioning(wl, 10)
    dense = G.dense_compare(gf, of, 1.0)
    assert max(dense.values()) <= TOL, dense
    rel = G.compare(gf, of)
    for k, v in rel.items():
        assert v <= max(TOL, 10.0 * sens[k]), (k, v, sens[k])


def test_relaxing_fluid_milne_pi_components():
    """All ten pi~ components nonzero (moving relaxing fluid in Milne coordinates)."""
    from . import analytic as A
    gr = ics.Grid(21, 5, 41, 0.1, 0.2, 0.05)
    ic = A.relaxing_fluid_milne(gr, 1.0, 10.0, 0.4, 0.6, A.conformal_taupi(10.0, 0.1))
    # rotate part of the x motion into y so that every component is populated
    ic["uy"] = 0.5 * ic["ux"]
    p = dict(nx=21, ny=5, ne=41, dx=0.1, dy=0.2, de=0.05, tau0=1.0, h=0.01, etas=0.1,
             viscous=1, cartesian=0)
    wl = W.Workload("relaxing_fluid_21x5x41", p, "conformal", 10, ic=ic)
    _both(wl, 10)


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 7), (5, 1, 1), (3, 4, 1)])
def test_degenerate_grids(shape):
    """Tiny and one-dimensional grids (uniform Bjorken state plus a bump)."""
    nx, ny, ne = shape
    gr = ics.Grid(nx, ny, ne, 0.3, 0.3, 0.3)
    ic = ics.bjorken(gr, 20.0, 0.5)
    ic["eps"] = ic["eps"] * (1.0 + 0.3 * np.random.default_rng(1).random(gr.shape))
    p = dict(nx=nx, ny=ny, ne=ne, dx=0.3, dy=0.3, de=0.3, tau0=0.6, h=0.01, etas=0.1,
             viscous=1, cartesian=0)
    wl = W.Workload(f"degenerate_{nx}x{ny}x{ne}", p, E.cached_synthetic_table(), 5, ic=ic)
    _both(wl, 5)


def test_all_vacuum():
    """Every cell below the cutoff: the state stays vacuum and nothing iterates."""
    gr = ics.Grid(9, 7, 5, 0.3, 0.3, 0.3)
    ic = dict(eps=np.full(gr.shape, 5e-8), ux=np.zeros(gr.shape), uy=np.zeros(gr.shape),
              ue=np.zeros(gr.shape))
    p = dict(nx=9, ny=7, ne=5, dx=0.3, dy=0.3, de=0.3, tau0=0.6, h=0.01, etas=0.1, viscous=1,
             cartesian=0)
    wl = W.Workload("vacuum_9x7x5", p, E.cached_synthetic_table(), 3, ic=ic)
    g, o, rel = _both(wl, 3)
    d = g.diag()
    assert d["vacuum"] == gr.ncell and d["solves"] == 0 and d["eps_max"] == 0.0


def test_cold_guess_matches_prev_guess():
    """The root-solve result does not depend on the starting guess (polish step)."""
    wl = W.hotspots_viscous(nx=33, ny=29, ne=7, dx=0.4, dy=0.4, de=0.5, steps=8, seed=6)
    _say("cold vs prev guess")
    import paper_1802_04449_amd as K
    a = G.run_gpu(wl, 8).fields()
    b = G.run_gpu(wl, 8, guess=K.KTMI_GUESS_COLD).fields()
    G.assert_parity(b, a, 1e-12, "cold vs prev")


def test_bitwise_deterministic():
    """Two runs of the same case are bitwise identical (no races, fixed reduction order)."""
    wl = W.hotspots_viscous(nx=37, ny=31, ne=9, dx=0.35, dy=0.35, de=0.4, steps=6, seed=7)
    _say("determinism")
    a = G.run_gpu(wl, 6)
    b = G.run_gpu(wl, 6)
    fa, fb = a.fields(), b.fields()
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
    assert a.diag() == b.diag()


def test_checkpoint_split_steps():
    """10 steps in one call equal 4 + 6 steps in two calls, bitwise."""
    wl = W.hotspots_viscous(nx=29, ny=27, ne=7, dx=0.4, dy=0.4, de=0.5, steps=10, seed=8)
    _say("split steps")
    a = G.run_gpu(wl, 10)
    b = G.run_gpu(wl, 4)
    b.step(6)
    fa, fb = a.fields(), b.fields()
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k


def test_hotspots_viscous_full_size_201x201x105():
    """The benchmark configuration at full size, in the launch configuration the
    benchmark times: 2 steps, compared over every cell."""
    wl = W.hotspots_viscous(steps=2)
    threads = min(16, os.cpu_count() or 1)
    _both(wl, 2, threads=threads)


def test_tile_shapes_bitwise_identical():
    """Every workgroup tile shape computes each face once with the same arithmetic,
    so the fields are bitwise identical whichever shape the launcher uses."""
    import paper_1802_04449_amd as K
    wl = W.hotspots_viscous(nx=27, ny=23, ne=19, dx=0.45, dy=0.45, de=0.4, steps=4, seed=9)
    _say("tile shapes")
    ref = None
    for t in range(K.ktmi_tile_count()):
        f = G.run_gpu(wl, 4, tile=t).fields()
        if ref is None:
            ref = f
            of = G.run_oracle(wl, 4).fields()
            G.assert_parity(f, of, TOL, "tile 0")
            continue
        for k in f:
            assert np.array_equal(f[k], ref[k]), (t, k)
