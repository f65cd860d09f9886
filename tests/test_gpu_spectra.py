"""Smooth Cooper-Frye spectra on the GPU (ktmi_spectra through the C ABI) against
the CPU oracle on the same surface records, and against the Bjorken closed form.

Both sides evaluate the same formula in FP64 with their own exp / cosh / sinh,
and the GPU adds the elements in slices, so the bar is 1e-12 of the species'
largest bin plus 1e-11 of the bin itself (not bit-identity)."""
import math
import sys

import numpy as np
import pytest

import oracle as O
from hydro_inputs import eos as E
from hydro_inputs import workloads as W

pytestmark = pytest.mark.gpu

SPECIES = ([0.13957, 0.49368, 0.93827], [1.0, 1.0, 2.0], [-1, -1, 1], [0.0, 0.0, 0.0])


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _bins(nY=5, npt=15, nphi=48):
    Y = np.linspace(-2.0, 2.0, nY)
    x, _ = np.polynomial.laguerre.laggauss(npt)
    pt = 0.35 * x  # Gauss-Laguerre nodes scaled to a 0.35 GeV slope
    u, _ = np.polynomial.legendre.leggauss(nphi)
    phi = math.pi * (u + 1.0)
    return Y, pt, phi


def _close(g, o, label):
    scale = np.abs(o).reshape(o.shape[0], -1).max(axis=1)[:, None, None, None]
    bad = np.abs(g - o) > 1e-12 * scale + 1e-11 * np.abs(o)
    rel = float((np.abs(g - o) / (scale + 1e-300)).max())
    _say(f"{label}: max dev / species scale {rel:.2e}")
    assert not bad.any(), (label, rel, np.argwhere(bad)[:5].tolist())


def _surface(wl, steps, ef, with_pi=True):
    import paper_1802_04449_amd as K
    h = K.Hydro(**wl.params)
    h.set_eos(wl.eos)
    h.set_initial(wl.ic)
    h.step(steps)
    tA = h.diag()["tau"]
    A = h.snapshot(with_pi)
    h.step(1)
    tB = h.diag()["tau"]
    B = h.snapshot(with_pi)
    return h.surface(A, tA, B, tB, ef)


@pytest.mark.parametrize("delta_f", [False, True])
def test_spectra_on_found_surface(delta_f):
    """Elements found by the GPU finder on a viscous hotspot run; pions, kaons,
    protons; 5 x 15 x 13 bins (13 phi bins: not a multiple of the per-thread 8)."""
    import paper_1802_04449_amd as K
    wl = W.hotspots_viscous(nx=41, ny=37, ne=11, dx=0.35, dy=0.35, de=0.4, steps=12, seed=21)
    _say(f"spectra on found surface delta_f={delta_f}")
    el = _surface(wl, 10, 0.5)
    assert el.shape[0] > 500
    Y, pt, phi = _bins(5, 15, 13)
    T, wP = 0.15, (0.7 if delta_f else 0.0)
    g = K.spectra(el, T, wP, SPECIES, Y, pt, phi).cpu().numpy()
    o = O.spectra(el.cpu().numpy(), T, wP, SPECIES, Y, pt, phi)
    assert np.abs(o).max() > 0
    _close(g, o, f"found surface delta_f={delta_f}")


def test_spectra_bjorken_closed_form():
    """Boost-invariant constant-tau elements at rest on the GPU against
    g tau/(2 pi hbarc)^3 sum_n (-sigma)^(n-1) 2 m_T K1(n m_T/T)."""
    import torch
    from scipy.special import kv

    import paper_1802_04449_amd as K
    _say("spectra Bjorken closed form")
    T, tau, deta = 0.15, 5.0, 0.01
    etas = np.arange(-12.0 + 0.5 * deta, 12.0, deta)
    el = np.zeros((etas.size, 24))
    el[:, 1] = tau
    el[:, 4] = etas
    el[:, 5] = tau * deta
    Y, pt, phi = np.array([0.0, 0.7]), np.array([0.2, 1.0, 2.5]), np.array([0.0, 1.3, 2.9])
    g = K.spectra(torch.tensor(el, device="cuda"), T, 0.0, SPECIES, Y, pt, phi).cpu().numpy()
    pref = 1.0 / (2.0 * math.pi * E.HBARC) ** 3
    for s, (m, d, st) in enumerate(zip(*SPECIES[:3])):
        for ip, p in enumerate(pt):
            mT = math.hypot(m, p)
            ref = d * tau * pref * sum((-st) ** (n - 1) * 2 * mT * kv(1, n * mT / T)
                                       for n in range(1, 61))
            assert np.max(np.abs(g[s, :, ip, :] / ref - 1.0)) < 1e-9, (s, ip)


def test_spectra_full_bins_sampled():
    """The paper's 41 x 15 x 48 bins on the benchmark grid's surface (41660
    elements, e_f = 0.3 GeV/fm^3, delta f on) for pions and protons; the oracle
    evaluates a sample of bins."""
    import paper_1802_04449_amd as K
    wl = W.hotspots_viscous(steps=11)
    _say("spectra full bins")
    el = _surface(wl, 10, 0.3)
    assert el.shape[0] > 10000
    Y, pt, phi = _bins(41, 15, 48)
    sp = ([0.13957, 0.93827], [1.0, 2.0], [-1, 1], [0.0, 0.0])
    T, wP = 0.137, 0.3 + 0.1
    g = K.spectra(el, T, wP, sp, Y, pt, phi).cpu().numpy()
    iy, ip, iq = [0, 20, 37], [0, 6, 14], [0, 11, 30, 47]
    o = O.spectra(el.cpu().numpy(), T, wP, sp, Y[iy], pt[ip], phi[iq])
    _close(g[:, iy][:, :, ip][:, :, :, iq], o, "full bins (sampled)")


def test_spectra_empty_surface():
    import torch

    import paper_1802_04449_amd as K
    Y, pt, phi = _bins(3, 4, 9)
    g = K.spectra(torch.zeros((0, 24), dtype=torch.float64, device="cuda"), 0.15, 0.0, SPECIES,
                  Y, pt, phi)
    assert float(g.abs().max()) == 0.0
