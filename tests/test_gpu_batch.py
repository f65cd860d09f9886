"""Graph replay and grouped (batched) stepping against single-event stepping.

A replayed graph and a grouped launch run the same per-cell arithmetic as the
plain path, so the fields must be bitwise identical; the plain path itself is
pinned to the oracle in test_gpu_parity.py (and once more here for one event)."""
import numpy as np
import pytest

from hydro_inputs import workloads as W

from . import gpu_common as G

pytestmark = pytest.mark.gpu


def _make(wl, stream, **kw):
    import paper_1802_04449_amd as K
    d = dict(wl.params)
    d.update(kw)
    h = K.Hydro(stream=stream, **d)
    h.set_eos(wl.eos)
    if wl.T4 is not None:
        h.set_initial_conserved(wl.T4)
    else:
        h.set_initial(wl.ic)
    return h


def _same(a, b, label):
    fa, fb = a.fields(), b.fields()
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), (label, k)


def test_graph_replay_matches_plain_steps():
    import torch
    print("[gpu-case] graph replay", flush=True)
    wl = W.hotspots_viscous(nx=37, ny=33, ne=11, dx=0.35, dy=0.35, de=0.4, steps=7, seed=12)
    st = torch.cuda.Stream()
    a = _make(wl, st)
    b = _make(wl, st)
    b.set_graph(True)
    a.step(7)
    b.step(3)
    b.step(4)  # odd counts exercise both buffer parities
    _same(a, b, "graph")
    assert a.diag() == b.diag()


def test_group_matches_single_events():
    import torch
    print("[gpu-case] grouped events", flush=True)
    sizes = [(41, 1, 0.08), (23, 17, 0.0), (31, 9, 0.16), (27, 1, 0.0), (35, 19, 0.08)]
    evs = W.event_batch(nev=len(sizes), sizes=sizes, steps=6)
    for wl in evs:  # small grids, same physics
        wl.params.update(dx=0.45, dy=0.45, de=0.45)
    st = torch.cuda.Stream()
    import paper_1802_04449_amd as K
    solo = [_make(wl, st) for wl in evs]
    grouped = [_make(wl, st) for wl in evs]
    for h in solo:
        h.step(6)
    grp = K.Group(grouped)
    assert grp.classes >= 3
    grp.step(2)
    grp.set_graph(True)
    grp.step(4)
    for e, (x, y) in enumerate(zip(solo, grouped)):
        _same(x, y, f"event {e}")
        assert x.diag() == y.diag(), e
    # one member against the oracle as well
    of = G.run_oracle(evs[2], 6).fields()
    G.assert_parity(grouped[2].fields(), of, 1e-12, "grouped event vs oracle")


def test_group_with_second_order_events():
    """A group mixing first-order events with lambda_1 events (different kernel
    classes in one step) gives the single-run fields bit for bit."""
    import torch
    print("[gpu-case] grouped lambda_1 events", flush=True)
    import paper_1802_04449_amd as K
    evs = W.event_batch(nev=3, seed0=80, steps=5, sizes=[(29, 7, 0.08), (25, 5, 0.16), (31, 9, 0.08)])
    for wl in evs:
        wl.params.update(dx=0.45, dy=0.45, de=0.45)
    evs[0].params.update(lambda1_hat=-8.0, taupi_coef=6.0)
    evs[2].params.update(lambda1_hat=-12.0)
    st = torch.cuda.Stream()
    solo = [_make(wl, st) for wl in evs]
    grouped = [_make(wl, st) for wl in evs]
    for h in solo:
        h.step(5)
    grp = K.Group(grouped)
    assert grp.classes >= 2
    grp.step(5)
    for e, (x, y) in enumerate(zip(solo, grouped)):
        _same(x, y, f"event {e}")
    of = G.run_oracle(evs[0], 5).fields()
    G.assert_parity(grouped[0].fields(), of, 1e-12, "grouped lambda_1 event vs oracle")


def test_autotuner_selects_a_tile_and_results_do_not_change():
    """The autotuner times every tile shape on the event and keeps the fastest;
    the state it then produces equals an untuned run's (any tile gives the same
    fields)."""
    import paper_1802_04449_amd as K
    from paper_1802_04449_amd import autotune
    print("[gpu-case] autotune", flush=True)
    wl = W.hotspots_viscous(nx=41, ny=37, ne=13, dx=0.35, dy=0.35, de=0.4, steps=4, seed=14)
    tuned = _make(wl, None)
    tile, times = autotune.tune(tuned, steps=1, repeats=1, use_cache=False)
    assert 0 <= tile < K.ktmi_tile_count() and K.ktmi_get_tile(tuned.h) == tile
    assert set(times) == set(range(K.ktmi_tile_count()))
    assert times[tile] == min(times.values())
    # restart from the initial state with the chosen tile, compare with the default tile
    tuned.set_initial(wl.ic)
    tuned.step(4)
    plain = _make(wl, None)
    plain.step(4)
    _same(tuned, plain, "autotuned tile")
