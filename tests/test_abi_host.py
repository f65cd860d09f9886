"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
function include/ktmi.h declares, and validates descriptors without touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ktmi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ktmi_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    import paper_1802_04449_amd as K
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(K.lib, n), n
        assert callable(getattr(K.lib, n))


def test_binding_names_match_abi():
    import paper_1802_04449_amd as K
    for n in _declared():
        if n in ("ktmi_kernel_count", "ktmi_kernel_name", "ktmi_last_error",
                 "ktmi_group_last_error"):
            continue
        assert hasattr(K, n), f"binding lacks {n}"


def _desc(**kw):
    import paper_1802_04449_amd as K
    d = K.ktmi_desc_default()
    for k, v in dict(nx=8, ny=8, ne=4, dx=0.3, dy=0.3, de=0.3, tau0=0.6, h=0.01).items():
        setattr(d, k, v)
    for k, v in kw.items():
        setattr(d, k, v)
    return d


def test_defaults_follow_the_paper():
    import paper_1802_04449_amd as K
    d = K.ktmi_desc_default()
    assert d.eps_cut == 1e-7  # energy-density cutoff of Sec. V.A
    assert d.newton_tol == 1e-12 and d.precision == K.KTMI_FP64
    assert d.taupi_coef == 5.0 and d.lambda1_hat == 0.0  # tau_pi = 5 eta/(sT), Sec. II
    assert d.zetas == 0.0 and d.baryon == 0  # no bulk pressure, no baryon density (Sec. III)
    assert d.taubulk_coef == 5.0


@pytest.mark.parametrize("bad", [dict(nx=0), dict(ne=-1), dict(dx=0.0), dict(h=-0.01),
                                 dict(tau0=0.0), dict(viscous=1, etas=0.0), dict(theta=2.5),
                                 dict(newton_maxit=0), dict(precision=7), dict(guess=9),
                                 dict(viscous=1, etas=0.1, taupi_coef=0.0),
                                 dict(lambda1_hat=float("nan")), dict(lambda1_hat=float("inf")),
                                 dict(zetas=0.05),  # bulk without viscous mode
                                 dict(baryon=1),  # baryon density without viscous mode
                                 dict(viscous=1, etas=0.1, zetas=-0.1),
                                 dict(viscous=1, etas=0.1, zetas=float("nan")),
                                 dict(viscous=1, etas=0.1, zetas=0.05, taubulk_coef=0.0),
                                 dict(viscous=1, etas=0.1, baryon=2),
                                 dict(viscous=1, etas=0.1, zetas=0.05, precision=1),
                                 dict(viscous=1, etas=0.1, baryon=1, lambda1_hat=-10.0)])
def test_invalid_descriptors_rejected(bad):
    import paper_1802_04449_amd as K
    d = _desc(**bad)
    with pytest.raises(K.KtmiError):
        K.ktmi_create(d)
    assert K.ktmi_workspace_bytes(d) == 0


def test_workspace_size_and_state_errors():
    import paper_1802_04449_amd as K
    d = _desc(viscous=1, etas=0.1)
    n = K.ktmi_workspace_bytes(d)
    assert n >= 39 * 8 * 8 * 4 * 8
    h = K.ktmi_create(d)
    try:
        with pytest.raises(K.KtmiError, match="initial state"):
            K.ktmi_step(h, 1)
        with pytest.raises(K.KtmiError, match="no workspace"):
            K.ktmi_set_initial_primitive(h, 1, 1, 1, 1)
        with pytest.raises(K.KtmiError, match="aligned"):
            K.ktmi_bind(h, 8, n, 0)
        with pytest.raises(K.KtmiError, match="smaller"):
            K.ktmi_bind(h, 256, n - 8, 0)
    finally:
        K.ktmi_destroy(h)


def test_bulk_workspace_holds_four_more_fields():
    import paper_1802_04449_amd as K
    d0 = _desc(viscous=1, etas=0.1)
    d1 = _desc(viscous=1, etas=0.1, zetas=0.05, baryon=1)
    n = 8 * 8 * 4  # cells of _desc, padded to 32
    assert K.ktmi_workspace_bytes(d1) - K.ktmi_workspace_bytes(d0) == 4 * ((n + 31) // 32 * 32) * 8


def test_tile_shapes_cover_256_threads():
    import paper_1802_04449_amd as K
    n = K.ktmi_tile_count()
    assert n >= 4
    for t in range(n):
        tx, ty, tz = K.ktmi_tile_shape(t)
        assert tx * ty * tz == 256
    with pytest.raises(K.KtmiError):
        K.ktmi_tile_shape(n)
    d = _desc(nx=50, ny=40, ne=1)
    h = K.ktmi_create(d)
    try:
        tx, ty, tz = K.ktmi_tile_shape(K.ktmi_get_tile(h))
        assert tz == 1  # a boost-invariant grid gets a flat tile automatically
        K.ktmi_set_tile(h, 0)
        assert K.ktmi_get_tile(h) == 0
        with pytest.raises(K.KtmiError):
            K.ktmi_set_tile(h, n)
    finally:
        K.ktmi_destroy(h)


def test_group_workspace_size():
    import paper_1802_04449_amd as K
    assert K.ktmi_group_workspace_bytes(0) == 0
    assert K.ktmi_group_workspace_bytes(64) > 64 * 400


def test_learned_guess_argument_checks():
    """Network entry points reject bad arguments before touching a device."""
    import paper_1802_04449_amd as K
    assert K.ktmi_mlp_nparam() == 1249
    assert K.ktmi_mlp_grad_workspace_bytes(0) == 0
    assert K.ktmi_mlp_grad_workspace_bytes(1) >= (1249 + 2) * 4
    # the gradient workspace stops growing once every workgroup sweeps several chunks
    assert K.ktmi_mlp_grad_workspace_bytes(10 ** 7) == K.ktmi_mlp_grad_workspace_bytes(10 ** 6)
    lib = K.lib
    assert lib.ktmi_mlp_forward(None, 4, None, None, 1e-7, None, 0, None) == K.KTMI_EINVAL
    assert lib.ktmi_mlp_forward(8, 0, None, None, 1e-7, None, 0, None) == K.KTMI_OK  # empty input
    assert lib.ktmi_mlp_forward(8, 4, 8, 8, 1e-7, 8, 7, None) == K.KTMI_EINVAL        # bad mode
    assert lib.ktmi_mlp_grad(8, 0, 8, 8, 8, 1e-7, 0, 8, 8, 1 << 20, None) == K.KTMI_EINVAL
    assert lib.ktmi_mlp_grad(8, 1000, 8, 8, 8, 1e-7, 0, 8, 8, 16, None) == K.KTMI_EINVAL  # short ws
    assert lib.ktmi_mlp_grad_noalloc(8, 0, 8, 8, 8, 1e-7, 0, 8, None) == K.KTMI_EINVAL  # empty
    assert lib.ktmi_mlp_grad_noalloc(8, 2 ** 31 - 128, 8, 8, 8, 1e-7, 0, 8,
                                     None) == K.KTMI_EINVAL                          # too many
    assert lib.ktmi_mlp_grad_noalloc(8, 100, 8, 8, 8, 1e-7, 5, 8, None) == K.KTMI_EINVAL  # mode
    assert lib.ktmi_mlp_grad_noalloc(8, 100, None, 8, 8, 1e-7, 0, 8, None) == K.KTMI_EINVAL
    assert lib.ktmi_mlp_adam(8, 8, 8, 8, 0, 1e-3, 0.9, 0.999, 1e-8, None) == K.KTMI_EINVAL  # t < 1
    assert lib.ktmi_mlp_adam(8, 8, 8, 8, 1, 1e-3, 1.0, 0.999, 1e-8, None) == K.KTMI_EINVAL  # b1 = 1
    d = _desc(guess=K.KTMI_GUESS_MLP)
    h = K.ktmi_create(d)  # the mode is accepted; the parameters are checked at set-up
    try:
        with pytest.raises(K.KtmiError, match="bind"):
            K.ktmi_set_mlp(h, 8, K.KTMI_MLP_FP32)
        with pytest.raises(K.KtmiError, match="unknown guess"):
            K.ktmi_set_guess(h, 5)
        with pytest.raises(K.KtmiError, match="ktmi_set_mlp"):
            K.ktmi_set_guess(h, K.KTMI_GUESS_MLP)
        K.ktmi_set_guess(h, K.KTMI_GUESS_COLD)
        with pytest.raises(K.KtmiError, match="no state"):
            K.ktmi_harvest(h, 8, 8, 8)
    finally:
        K.ktmi_destroy(h)


def test_freezeout_and_spectra_argument_checks():
    """Surface, stop and spectra entry points reject bad arguments before touching
    a device (a handle without a workspace, short workspaces, bad statistics)."""
    import ctypes as C

    import numpy as np

    import paper_1802_04449_amd as K
    lib = K.lib
    h = K.ktmi_create(_desc())
    try:
        assert K.ktmi_snapshot_doubles(h, False) == 4 * 8 * 8 * 4
        assert K.ktmi_snapshot_doubles(h, True) == 14 * 8 * 8 * 4
        taken = C.c_int()
        assert lib.ktmi_step_until(h, 1.0, -1, 1, C.byref(taken)) == K.KTMI_EINVAL
        assert lib.ktmi_step_until(h, 1.0, 5, 0, C.byref(taken)) == K.KTMI_EINVAL
        assert lib.ktmi_step_until(h, 1.0, 5, 1, None) == K.KTMI_EINVAL
        # no slices, reversed times, a non-finite threshold, then no workspace
        assert lib.ktmi_surface(h, None, 1.0, 8, 2.0, 0, 0.3, 8, 4, 8) == K.KTMI_EINVAL
        assert lib.ktmi_surface(h, 8, 2.0, 8, 1.0, 0, 0.3, 8, 4, 8) == K.KTMI_EINVAL
        assert lib.ktmi_surface(h, 8, 1.0, 8, 2.0, 0, float("nan"), 8, 4, 8) == K.KTMI_EINVAL
        assert lib.ktmi_surface(h, 8, 1.0, 8, 2.0, 0, 0.3, None, 4, 8) == K.KTMI_EINVAL
        assert lib.ktmi_surface(h, 8, 1.0, 8, 2.0, 0, 0.3, 8, 4, 8) == K.KTMI_ESTATE
    finally:
        K.ktmi_destroy(h)
    assert K.ktmi_spectra_workspace_bytes(-1, 1, 1, 1, 1) == 0
    assert K.ktmi_spectra_workspace_bytes(100, 0, 1, 1, 1) == 0
    nb = K.ktmi_spectra_workspace_bytes(1000, 2, 41, 15, 48)
    assert nb >= 2 * 41 * 15 * 48 * 8
    args = dict(mass=[0.14, 0.94], dof=[1, 2], stat=[-1, 1], mu=[0, 0], Y=np.zeros(41),
                pt=np.ones(15), phi=np.ones(48))

    def call(**kw):
        a = dict(args)
        a.update(kw)
        try:
            K.ktmi_spectra(8, kw.pop("n", 1000), kw.pop("T", 0.15), 0.0, a["mass"], a["dof"],
                           a["stat"], a["mu"], a["Y"], a["pt"], a["phi"], 8, 8,
                           kw.pop("ws_bytes", nb), 0)
        except K.KtmiError as e:
            return str(e)
        return "ok?"

    assert "failed" in call(ws_bytes=nb - 8)          # short workspace
    assert "failed" in call(T=0.0)                    # T must be > 0
    assert "failed" in call(stat=[-1, 2])             # statistics in {-1, 0, 1}
    assert "failed" in call(mass=[0.14, -1.0])        # negative mass
