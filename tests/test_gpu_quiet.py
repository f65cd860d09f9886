"""Quiet-tile skipping against the full computation: a step that skips tiles
whose 6-cell neighbourhood was vacuum after the previous step must give the
same fields and diagnostics bit for bit, also while matter expands into
skipped regions (tiles waking up), in ideal and viscous mode, Milne and
Cartesian coordinates, grouped and graph-replayed."""
import numpy as np
import pytest

from hydro_inputs import eos as EOS
from hydro_inputs import workloads as W

from . import gpu_common as G

pytestmark = pytest.mark.gpu


def _run(wl, steps, quiet, stream=None, **kw):
    import paper_1802_04449_amd as K
    d = dict(wl.params)
    d.update(kw)
    h = K.Hydro(stream=stream, **d)
    h.set_eos(wl.eos)
    h.set_quiet_skip(quiet)
    h.set_initial(wl.ic)
    h.step(steps)
    return h


def _same(a, b, label):
    fa, fb = a.fields(), b.fields()
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), (label, k)
    assert a.diag() == b.diag(), (label, a.diag(), b.diag())


@pytest.mark.parametrize("viscous,cartesian", [(1, 0), (0, 0), (1, 1)])
def test_quiet_skip_matches_full_computation(viscous, cartesian):
    """An expanding fireball on a grid with a wide vacuum margin: 150 steps
    (1.5 fm/c) move the edge across several tile boundaries."""
    import paper_1802_04449_amd as K
    print(f"[gpu-case] quiet skip viscous={viscous} cartesian={cartesian}", flush=True)
    wl = W.hotspots_viscous(nx=61, ny=61, ne=9, dx=0.35, dy=0.35, de=0.5, steps=150, seed=31)
    kw = dict(viscous=viscous, cartesian=cartesian)
    if not viscous:
        kw["etas"] = 0.0
    a = _run(wl, 150, False, **kw)
    b = _run(wl, 150, True, **kw)
    _same(a, b, f"quiet skip v{viscous} c{cartesian}")
    q, n = K.ktmi_quiet_tiles(b.h)
    assert 0 < q < n, (q, n)


@pytest.mark.parametrize("kw", [dict(lambda1_hat=-10.0, taupi_coef=7.5), dict(precision=1)])
def test_quiet_skip_second_order_and_mixed(kw):
    """Skipping with the lambda_1 kernels and with the mixed-precision kernels:
    bitwise equal to the same variant without skipping."""
    print(f"[gpu-case] quiet skip {kw}", flush=True)
    wl = W.hotspots_viscous(nx=61, ny=61, ne=9, dx=0.35, dy=0.35, de=0.5, steps=100, seed=33)
    a = _run(wl, 100, False, **kw)
    b = _run(wl, 100, True, **kw)
    _same(a, b, f"quiet skip {kw}")


def test_quiet_skip_grouped_graph():
    """Three events (one ideal) stepped as a group replayed from a graph, with
    skipping on, against plain single runs without it."""
    import torch
    import paper_1802_04449_amd as K
    print("[gpu-case] quiet skip group graph", flush=True)
    evs = W.event_batch(nev=3, seed0=70, steps=40,
                        sizes=[(45, 9, 0.08), (41, 1, 0.0), (43, 7, 0.16)])
    st = torch.cuda.Stream()
    hs = []
    for wl in evs:
        h = K.Hydro(stream=st, **wl.params)
        h.set_eos(wl.eos)
        h.set_quiet_skip(True)
        h.set_initial(wl.ic)
        hs.append(h)
    grp = K.Group(hs)
    grp.set_graph(True)
    grp.step(40)
    torch.cuda.synchronize()
    for wl, h in zip(evs, hs):
        ref = _run(wl, 40, False)
        _same(h, ref, wl.name)


def test_quiet_skip_needs_zero_pressure_at_zero_energy():
    import paper_1802_04449_amd as K
    wl = W.hotspots_viscous(nx=21, ny=21, ne=5, dx=0.5, dy=0.5, de=0.5, steps=1, seed=32)
    h = K.Hydro(**wl.params)
    t = EOS.cached_synthetic_table()
    P = np.array(t.P, dtype=np.float64)
    P[0] = 1e-3
    K.ktmi_set_eos_table(h.h, t.eps0, t.deps, P, t.T, t.cs2)
    with pytest.raises(K.KtmiError, match="P\\(0\\) = 0"):
        h.set_quiet_skip(True)
    h.set_eos(t)  # P(0) = 0 again
    h.set_quiet_skip(True)
    with pytest.raises(K.KtmiError, match="P\\(0\\) = 0"):
        K.ktmi_set_eos_table(h.h, t.eps0, t.deps, P, t.T, t.cs2)
