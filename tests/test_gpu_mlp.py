"""Learned root-solve guess on the GPU, through the C ABI: forward, gradient and
Adam kernels against the FP64 reference network, harvest of training samples,
the guess inside the step (parity with the oracle and with the previous-stage
guess), and the iteration count it saves."""
import json
import math
import os
import sys

import numpy as np
import pytest

import oracle as O
from hydro_inputs import eos as EOS
from hydro_inputs import ics
from hydro_inputs import workloads as W

from . import gpu_common as G

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _report(name, data):
    d = os.environ.get("KTMI_REPORT_DIR")
    if d and os.path.isdir(d):
        with open(os.path.join(d, f"{name}.json"), "w") as f:
            json.dump(data, f, indent=1)
    _say(f"{name}: {data}")


def _samples(n, seed, emin_frac=0.0):
    """(E, M, e) of random fluid states under the synthetic table EoS: e
    log-uniform in [1e-6, 60], |v| uniform in [0, 0.99]; the target e is the
    exact root of its own K."""
    eps, u = ics.random_states(n, seed, eps_lo=1e-6, eps_hi=60.0, vmax=0.99)
    o = O.Oracle(O.Params(2, 2, 2, 0.1, 0.1, 0.1, tau0=1.0, h=0.01),
                 eos=EOS.cached_synthetic_table())
    K = o.prim2K(eps, u)
    return K[:, 0].copy(), np.linalg.norm(K[:, 1:], axis=1), eps


def _params(seed, scale=0.4):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, O.mlp_nparam()).astype(np.float32)


def _dev(a, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def _forward(p32, E, M, mode, emin=1e-7):
    import torch
    import paper_1802_04449_amd as K
    pt, Et, Mt = _dev(p32), _dev(E), _dev(M)
    g = torch.empty_like(Et)
    K.ktmi_mlp_forward(pt.data_ptr(), E.size, Et.data_ptr(), Mt.data_ptr(), emin, g.data_ptr(),
                       mode, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return g.cpu().numpy()


def _grad(p32, E, M, eps, mode, emin=1e-7):
    import torch
    import paper_1802_04449_amd as K
    pt, Et, Mt, et = _dev(p32), _dev(E), _dev(M), _dev(eps)
    n = E.size
    nb = K.ktmi_mlp_grad_workspace_bytes(n)
    ws = torch.empty(nb // 4 + 64, dtype=torch.float32, device="cuda")
    out = torch.zeros(K.ktmi_mlp_nparam() + 2, dtype=torch.float32, device="cuda")
    K.ktmi_mlp_grad(pt.data_ptr(), n, Et.data_ptr(), Mt.data_ptr(), et.data_ptr(), emin, mode,
                    out.data_ptr(), ws.data_ptr(), nb, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    return o[:-2].astype(np.float64), float(o[-2]), float(o[-1])


@pytest.mark.parametrize("mode,tol", [(0, 5e-6), (1, 2e-2)])
def test_forward_matches_reference(mode, tol):
    """FP32 per-lane forward within 5e-6 E of the FP64 network; the BF16
    matrix-core forward (rounded W2 and hidden layer) within 2e-2 E.  5003
    samples: 20 workgroups of 256, ragged tail."""
    _say(f"mlp forward mode={mode}")
    E, M, eps = _samples(5003, 1)
    p = _params(2)
    g = _forward(p, E, M, mode)
    ref = O.mlp_forward(p.astype(np.float64), E, M)
    err = np.abs(g - ref) / E
    lo = np.maximum(0.0, E - M * M / E)
    assert np.all(g >= lo * (1 - 1e-15)) and np.all(g <= E)
    assert err.max() <= tol, err.max()
    if mode == 1:  # the matrix-core path must not just fall back to something crude
        assert np.median(err) <= tol / 4


def test_forward_below_emin_returns_E():
    E, M, _ = _samples(300, 3)
    E[::3] = 1e-9
    g = _forward(_params(4), E, M, 1, emin=1e-7)
    np.testing.assert_array_equal(g[::3], E[::3])


@pytest.mark.parametrize("mode,tol,n", [(0, 1e-5, 3001), (0, 1e-5, 70001), (1, 2e-2, 3001)])
def test_gradient_matches_reference(mode, tol, n):
    """FP32 backward (per-workgroup LDS folds, fixed-order cross-workgroup fold)
    vs the FP64 gradient: 1e-5 of max |g| with the FP32 forward, 2e-2 with the
    BF16 forward.  n = 70001 runs every workgroup over several chunks."""
    _say(f"mlp grad mode={mode} n={n}")
    E, M, eps = _samples(n, 5)
    p = _params(6)
    g, loss, cnt = _grad(p, E, M, eps, mode)
    L, ref = O.mlp_loss_grad(p.astype(np.float64), E, M, eps)
    assert cnt == n
    err = np.abs(g - ref).max() / np.abs(ref).max()
    assert err <= tol, err
    assert loss == pytest.approx(L, rel=tol)


def test_gradient_skips_samples_below_emin():
    E, M, eps = _samples(4000, 7)
    E[5::9] = 1e-12
    p = _params(8)
    g, loss, cnt = _grad(p, E, M, eps, 0, emin=1e-7)
    keep = E >= 1e-7
    L, ref = O.mlp_loss_grad(p.astype(np.float64), E[keep], M[keep], eps[keep])
    assert cnt == keep.sum()
    assert np.abs(g - ref).max() / np.abs(ref).max() <= 1e-5
    assert loss == pytest.approx(L, rel=1e-5)


def test_gradient_bitwise_deterministic():
    E, M, eps = _samples(20000, 9)
    p = _params(10)
    a = _grad(p, E, M, eps, 1)
    b = _grad(p, E, M, eps, 1)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]


def test_adam_matches_reference():
    import torch
    import paper_1802_04449_amd as K
    rng = np.random.default_rng(11)
    n = K.ktmi_mlp_nparam()
    p = rng.normal(size=n).astype(np.float32)
    g = rng.normal(size=n).astype(np.float32)
    m = (0.1 * rng.normal(size=n)).astype(np.float32)
    v = (0.1 * rng.random(size=n)).astype(np.float32)
    pt, gt, mt, vt = (_dev(x) for x in (p, g, m, v))
    K.ktmi_mlp_adam(pt.data_ptr(), gt.data_ptr(), mt.data_ptr(), vt.data_ptr(), 3, 1e-2, 0.9,
                    0.999, 1e-8, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    pr, mr, vr = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    # the kernel receives the hyper-parameters as FP32 values: give the reference the same
    f32 = lambda x: float(np.float32(x))
    O.mlp_adam(pr, g.astype(np.float64), mr, vr, 3, lr=f32(1e-2), b1=f32(0.9), b2=f32(0.999),
               epsilon=f32(1e-8))
    # FP32 update: a few ulps of parameters of size ~1
    np.testing.assert_allclose(pt.cpu().numpy(), pr, rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(mt.cpu().numpy(), mr, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(vt.cpu().numpy(), vr, rtol=1e-6, atol=1e-7)


def test_harvest_matches_state():
    """E = T~^{tau tau}/tau - pi~^{tau tau}, M = |T~^{tau i}/tau - pi~^{tau i}|, e."""
    wl = W.hotspots_viscous(nx=23, ny=21, ne=7, dx=0.5, dy=0.5, de=0.6, steps=3, seed=12)
    g = G.run_gpu(wl, 3)
    E, M, e = (t.cpu().numpy() for t in g.harvest())
    f = g.fields()
    tau = g.diag()["tau"]
    K = [f[f"T{m}"].reshape(-1) / tau - f[f"pi{m}"].reshape(-1) for m in range(4)]
    np.testing.assert_allclose(E, K[0], rtol=1e-14, atol=1e-300)
    np.testing.assert_allclose(M, np.sqrt(K[1] ** 2 + K[2] ** 2 + K[3] ** 2), rtol=1e-14,
                               atol=1e-300)
    np.testing.assert_array_equal(e, f["eps"].reshape(-1))


# ---- the guess inside the step ------------------------------------------------
def _train(seed_list, grid, steps_at=(0, 4, 8), train_steps=1500, mode=0):
    import paper_1802_04449_amd as K
    from paper_1802_04449_amd import mlp
    states = []
    for s in seed_list:
        wl = W.hotspots_viscous(steps=max(steps_at), seed=s, **grid)
        g = G.run_gpu(wl, 0)
        done = 0
        for t in steps_at:
            g.step(t - done)
            done = t
            states.append(g.harvest())
    E, M, e = mlp.samples_from_states(states, emin=1e-7, seed=1)
    tr = mlp.Trainer(E, M, e, mode=mode, seed=3)
    L0 = tr.loss()
    tr.train(train_steps, batch=4096, lr=3e-3, lr_final=3e-4)
    return tr, L0, tr.loss(), E.size


def _run_with_guess(wl, steps, guess, params=None, mode=0):
    import paper_1802_04449_amd as K
    g = K.Hydro(**dict(wl.params, guess=guess))
    g.set_eos(wl.eos)
    if params is not None:
        g.set_mlp(params, mode)  # before the initial state: its root solve uses the guess too
    g.set_initial(wl.ic)
    g.step(steps)
    return g


GRID = dict(nx=61, ny=57, ne=15, dx=0.25, dy=0.25, de=0.4)


@pytest.fixture(scope="module")
def trained():
    _say("mlp training on harvested states")
    tr, L0, L1, n = _train([21, 22], GRID)
    _report("mlp_training", dict(samples=n, loss_initial=L0, loss_final=L1))
    assert L1 < 0.05 * L0, (L0, L1)
    return tr


@pytest.mark.parametrize("mode", [0, 1])
def test_learned_guess_matches_oracle(trained, mode):
    """Same results as the oracle (which starts from the previous stage) at the
    FP64 bar: the solve's result does not depend on its start."""
    import paper_1802_04449_amd as K
    wl = W.hotspots_viscous(steps=6, seed=23, **GRID)
    _say(f"learned guess parity mode={mode}")
    g = _run_with_guess(wl, 6, K.KTMI_GUESS_MLP, trained.params, mode)
    o = G.run_oracle(wl, 6)
    G.assert_parity(g.fields(), o.fields(), 1e-12, f"mlp guess mode {mode}")
    d = g.diag()
    assert d["nonconv"] == 0 and d["nans"] == 0


def test_learned_guess_saves_iterations(trained):
    """Held-out event: mean root-solve iterations (including the polish step)
    with the network's start vs the cold start (E) and the previous stage's e.
    The network starts the predictor's solves; the corrector's start from the
    predictor's e in every mode.  Measured on this case: prev 3.46, cold 3.62,
    network 3.22 (FP32 and BF16)."""
    import paper_1802_04449_amd as K
    wl = W.hotspots_viscous(steps=10, seed=24, **GRID)
    _say("learned guess gain")
    res = {}
    fields = {}
    for name, guess, params, mode in [("prev", K.KTMI_GUESS_PREV, None, 0),
                                      ("cold", K.KTMI_GUESS_COLD, None, 0),
                                      ("mlp_fp32", K.KTMI_GUESS_MLP, trained.params, 0),
                                      ("mlp_bf16", K.KTMI_GUESS_MLP, trained.params, 1)]:
        g = _run_with_guess(wl, 10, guess, params, mode)
        d = g.diag()
        res[name] = dict(newton_mean=d["newton_mean"], newton_max=d["newton_max"],
                         fallbacks=d["fallbacks"], solves=d["solves"])
        fields[name] = g.fields()
    _report("mlp_gain_hotspots_61x57x15", res)
    for name in ("cold", "mlp_fp32", "mlp_bf16"):
        G.assert_parity(fields[name], fields["prev"], 1e-12, f"{name} vs prev")
    for name in ("mlp_fp32", "mlp_bf16"):
        assert res[name]["newton_mean"] <= res["cold"]["newton_mean"] - 0.3, res
        assert res[name]["newton_mean"] < res["prev"]["newton_mean"], res


def test_batched_learned_mixed_matches_oracle(trained):
    """The combined path: uneven events stepped as one group, mixed precision,
    root solves started from the network (BF16 forward); each event within the
    reduced-precision bar (1e-6 in e and u~, L2 and hydro-cell max norms) of the
    FP64 oracle."""
    import torch
    import paper_1802_04449_amd as K
    evs = W.event_batch(nev=3, seed0=40, steps=6,
                        sizes=[(41, 9, 0.08), (35, 1, 0.16), (39, 7, 0.0)])
    st = torch.cuda.Stream()
    hs = []
    for wl in evs:
        h = K.Hydro(stream=st, precision=K.KTMI_MIXED, guess=K.KTMI_GUESS_MLP, **wl.params)
        h.set_eos(wl.eos)
        h.set_mlp(trained.params, K.KTMI_MLP_BF16)
        h.set_initial(wl.ic)
        hs.append(h)
    grp = K.Group(hs)
    _say(f"batched learned mixed: {grp.classes} classes")
    grp.step(6)
    torch.cuda.synchronize()
    for wl, h in zip(evs, hs):
        err = G.precision_errors(h.fields(), G.run_oracle(wl, 6).fields())
        _say(f"{wl.name}: " + ", ".join(f"{k} l2 {err[k]['l2']:.1e} max {err[k]['max_hydro']:.1e}"
                                       for k in ("eps", "ux", "uy", "ue")))
        for k in ("eps", "ux", "uy", "ue"):
            assert err[k]["l2"] <= 1e-6 and err[k]["max_hydro"] <= 1e-6, (wl.name, k, err[k])
