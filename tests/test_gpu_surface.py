"""Freeze-out surface finder and the e_max-driven stop on the GPU, through the C ABI,
against the CPU oracle.

The finder's inputs are two slices; both sides receive the same slices (taken
from the GPU state, or built from the closed-form Gubser flow), so the
comparison isolates the finder.  The set of hypercubes with an element is an
integer result and must match exactly, in the same (hypercube) order; the
records are compared to 1e-12 of each column's scale (both sides evaluate the
same expressions in the same order without contraction, so they are expected to
agree bit for bit, which is reported)."""
import sys

import numpy as np
import pytest

import oracle as O
from hydro_inputs import eos as E
from hydro_inputs import ics
from hydro_inputs import workloads as W

from . import gpu_common as G

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _hydro(wl, **kw):
    import paper_1802_04449_amd as K
    d = dict(wl.params)
    d.update(kw)
    h = K.Hydro(**d)
    h.set_eos(wl.eos)
    if wl.T4 is not None:
        h.set_initial_conserved(wl.T4)
    else:
        h.set_initial(wl.ic)
    return h


def _compare(gel, oel, label):
    """gel: GPU records (any order); oel: oracle records (hypercube order)."""
    g = gel
    assert g.shape == oel.shape, (label, g.shape, oel.shape)
    assert np.array_equal(g[:, 0], oel[:, 0]), label
    if len(oel) == 0:
        return True
    scale = np.maximum(np.abs(oel).max(axis=0), 1e-300)
    rel = (np.abs(g - oel) / scale).max(axis=0)
    worst = int(np.argmax(rel))
    assert rel.max() <= TOL, (label, worst, float(rel.max()))
    bitwise = bool(np.array_equal(g, oel))
    _say(f"{label}: {len(oel)} elements, max rel {rel.max():.2e}, bitwise {bitwise}")
    return bitwise


def _gpu_surface(h, A, tA, B, tB, ef, capacity=None):
    return h.surface(A, tA, B, tB, ef, capacity=capacity).cpu().numpy()


@pytest.mark.parametrize("with_pi", [False, True])
def test_surface_on_hydro_slices(with_pi):
    """Slices of a viscous hotspot run (ragged 41x37x11 grid) two steps apart."""
    wl = W.hotspots_viscous(nx=41, ny=37, ne=11, dx=0.35, dy=0.35, de=0.4, steps=12, seed=21)
    _say(f"surface on hydro slices with_pi={with_pi}")
    h = _hydro(wl)
    h.step(10)
    tA = h.diag()["tau"]
    A = h.snapshot(with_pi)
    h.step(2)
    tB = h.diag()["tau"]
    B = h.snapshot(with_pi)
    for ef in (0.5, 3.0):
        gel = _gpu_surface(h, A, tA, B, tB, ef)
        oel = O.surface(h.shape, (wl.params["dx"], wl.params["dy"], wl.params["de"]),
                        A.cpu().numpy(), tA, B.cpu().numpy(), tB, ef)
        assert len(oel) > 100
        _compare(gel, oel, f"hydro slices ef={ef} pi={with_pi}")


@pytest.mark.parametrize("ne,cart", [(1, False), (9, False), (9, True)])
def test_surface_on_gubser_slices(ne, cart):
    """Closed-form ideal Gubser slices uploaded as snapshots: a boost-invariant grid
    (one eta cell), a 3D grid, and the Cartesian measure."""
    import torch

    import paper_1802_04449_amd as K
    _say(f"surface on Gubser slices ne={ne} cart={cart}")
    n, dx = 45, 0.2
    g = ics.Grid(n, n, ne, dx, dx, 0.3)
    h = K.Hydro(nx=n, ny=n, ne=ne, dx=dx, dy=dx, de=0.3, tau0=1.0, h=0.05, cartesian=int(cart))
    eps_peak = E.C_SB * 0.4 ** 4

    def slice_at(t):
        X, Y, _ = g.mesh()
        e, ux, uy = ics.gubser_profile(X, Y, t, q=1.0, eps_peak_tau1=eps_peak)
        return np.stack([e, ux, uy, np.zeros_like(e)])

    tA, tB = 1.3, 1.35
    SA, SB = slice_at(tA), slice_at(tB)
    A = torch.tensor(SA, device="cuda")
    B = torch.tensor(SB, device="cuda")
    ef = 0.2 * eps_peak
    gel = _gpu_surface(h, A, tA, B, tB, ef)
    oel = O.surface((n, n, ne), (dx, dx, 0.3), SA, tA, SB, tB, ef, cartesian=cart)
    assert len(oel) > 50
    _compare(gel, oel, f"gubser slices ne={ne} cart={cart}")


def test_surface_capacity_and_empty_cases():
    import torch
    wl = W.hotspots_viscous(nx=33, ny=31, ne=7, dx=0.35, dy=0.35, de=0.4, steps=4, seed=22)
    _say("surface capacity / empty")
    h = _hydro(wl)
    h.step(2)
    tA = h.diag()["tau"]
    A = h.snapshot(False)
    h.step(2)
    tB = h.diag()["tau"]
    B = h.snapshot(False)
    sp = (wl.params["dx"], wl.params["dy"], wl.params["de"])
    oel = O.surface(h.shape, sp, A.cpu().numpy(), tA, B.cpu().numpy(), tB, 1.0)
    n = len(oel)
    assert n > 100
    # a buffer for a third of the elements: the count is still exact, and the
    # records written are the oracle's first ones
    import paper_1802_04449_amd as K
    cap = n // 3
    out = torch.full((cap, K.KTMI_SURF_REC), -7.0, dtype=torch.float64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    K.ktmi_surface(h.h, A.data_ptr(), tA, B.data_ptr(), tB, False, 1.0, out.data_ptr(), cap,
                   cnt.data_ptr())
    torch.cuda.synchronize()
    assert int(cnt.item()) == n
    got = out.cpu().numpy()
    assert np.array_equal(got[:, 0], oel[:cap, 0])
    assert np.allclose(got, oel[:cap], rtol=0, atol=1e-12 * np.abs(oel).max())
    # thresholds above and below every value: no element
    assert len(_gpu_surface(h, A, tA, B, tB, 1e6)) == 0
    assert len(_gpu_surface(h, A + 1.0, tA, B + 1.0, tB, 0.5)) == 0
    # capacity 0 only counts
    K.ktmi_surface(h.h, A.data_ptr(), tA, B.data_ptr(), tB, False, 1.0, 0, 0, cnt.data_ptr())
    torch.cuda.synchronize()
    assert int(cnt.item()) == n
    with pytest.raises(K.KtmiError):
        K.ktmi_surface(h.h, A.data_ptr(), tB, B.data_ptr(), tA, False, 1.0, out.data_ptr(), cap,
                       cnt.data_ptr())


def test_surface_full_size_201x201x105():
    """The benchmark grid, slices after 10 and 11 steps, every element against the
    oracle (the launch the benchmark times)."""
    wl = W.hotspots_viscous(steps=11)
    _say("surface full size")
    h = _hydro(wl)
    h.step(10)
    tA = h.diag()["tau"]
    A = h.snapshot(True)
    h.step(1)
    tB = h.diag()["tau"]
    B = h.snapshot(True)
    gel = _gpu_surface(h, A, tA, B, tB, 0.3)
    oel = O.surface(h.shape, (wl.params["dx"], wl.params["dy"], wl.params["de"]),
                    A.cpu().numpy(), tA, B.cpu().numpy(), tB, 0.3)
    assert len(oel) > 10000
    _compare(gel, oel, "full size")


def test_step_until_matches_oracle_stop():
    """The e_max-driven stop: the number of steps until e_max < e_stop equals the
    step at which the oracle's own e_max first falls below it."""
    wl = W.hotspots_viscous(nx=25, ny=23, ne=5, dx=0.5, dy=0.5, de=0.5, steps=60, seed=23)
    _say("step_until")
    o = G.run_oracle(wl, 0)
    emax = []
    for _ in range(60):
        o.step(1)
        emax.append(o.diag()["eps_max"])
    e_stop = 0.5 * (emax[0] + emax[-1])
    expect = next(i + 1 for i, v in enumerate(emax) if v < e_stop)
    h = _hydro(wl)
    assert h.step_until(e_stop, 60, check_every=1) == expect
    h2 = _hydro(wl)
    taken = h2.step_until(e_stop, 60, check_every=4)
    assert taken == next(k for k in range(4, 61, 4) if emax[k - 1] < e_stop)
    h3 = _hydro(wl)
    assert h3.step_until(-1.0, 7, check_every=3) == 7
