"""The CPU oracle against what the paper and the mathematics fix.

Each pin (tests/pins.py) compares the oracle with a closed form, a library
integrator, an exact discrete identity or a symmetry; none compares the oracle
with itself or with the HIP library.
"""
import pytest

from . import pins


@pytest.mark.parametrize("name", list(pins.ALL_PINS))
def test_pin(name):
    ok, info = pins.ALL_PINS[name]()
    assert ok, f"{name}: {info}"


def test_viscous_gubser_closed_form_matches_weyl_map():
    """The closed-form viscous Gubser state used by the gubser_viscous pin against
    the de Sitter-frame solution mapped back by automatic differentiation of the
    coordinate change (two independent routes), and its transversality and
    tracelessness."""
    import numpy as np

    from hydro_inputs import ics

    from . import analytic as A
    L, lam, e0 = 2.0, -10.0, 3.7
    g = np.array([1.0, -1.0, -1.0, -1.0])
    idx = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3)]
    for X in [(1.0, 0.3, -0.7, 0.0), (1.6, 2.1, 1.3, 0.4), (0.8, -3.0, 0.2, -1.0), (2.5, 0.05, 4.0, 0.0)]:
        e, ux, uy, pi, u = A.gubser_viscous_by_weyl(X, L, lam, e0)
        e2, ux2, uy2, pi2 = ics.gubser_viscous_profile(X[1], X[2], X[0], L, lam, e0)
        assert abs(e / e2 - 1.0) < 1e-13
        assert abs(ux - ux2) < 1e-13 and abs(uy - uy2) < 1e-13
        assert np.max(np.abs(pi - pi2)) < 1e-13 * np.max(np.abs(pi))
        ut = np.array([np.sqrt(1 + ux2 ** 2 + uy2 ** 2), ux2, uy2, 0.0])
        P = np.zeros((4, 4))
        for m, (a, b) in enumerate(idx):
            P[a, b] = P[b, a] = pi2[m]
        assert np.max(np.abs(P @ (g * ut))) < 1e-13 * np.max(np.abs(P))
        assert abs(np.sum(g * np.diag(P))) < 1e-13 * np.max(np.abs(P))
        # the Sec. V.C ratio pi~^{eta eta} / e = 2 / lambda1_hat holds everywhere
        assert abs(pi2[9] / e2 - 2.0 / lam) < 1e-13
