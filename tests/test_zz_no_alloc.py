"""The allocation-free gradient entry point (ktmi_mlp_grad_noalloc) against the
workspace one (ktmi_mlp_grad), through the C ABI: two calls in a row on one
GPU, the second with fewer samples (so fewer workgroup partials than the first
left in the shared scratch), in both forward modes.  The two entry points run
the same kernels and the same fixed-order fold, so the results must be equal
bit for bit."""
import numpy as np
import pytest

from hydro_inputs import ics

pytestmark = pytest.mark.gpu


def _samples(n, seed):
    # random fluid states turned into (E, M, e) by the conformal relation
    # T^{tau tau} = (e + P) u^tau u^tau - P, |T^{tau i}| = (e + P) u^tau |u|,
    # with P = e / 3: input generation only, no arithmetic of the method
    eps, u = ics.random_states(n, seed, eps_lo=1e-6, eps_hi=60.0, vmax=0.99)
    ut = np.sqrt(1.0 + np.sum(u * u, axis=1))
    w = eps * 4.0 / 3.0
    E = w * ut * ut - eps / 3.0
    M = w * ut * np.linalg.norm(u, axis=1)
    return E, M, eps


def _run(which, p32, E, M, eps, mode, emin=1e-7):
    import torch
    import paper_1802_04449_amd as K
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    pt, Et, Mt, et = dev(p32), dev(E), dev(M), dev(eps)
    n = E.size
    out = torch.full((K.ktmi_mlp_nparam() + 2,), float("nan"), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    if which == "ws":
        nb = K.ktmi_mlp_grad_workspace_bytes(n)
        ws = torch.empty(nb // 4 + 64, dtype=torch.float32, device="cuda")
        K.ktmi_mlp_grad(pt.data_ptr(), n, Et.data_ptr(), Mt.data_ptr(), et.data_ptr(), emin, mode,
                        out.data_ptr(), ws.data_ptr(), nb, stream)
    else:
        K.ktmi_mlp_grad_noalloc(pt.data_ptr(), n, Et.data_ptr(), Mt.data_ptr(), et.data_ptr(),
                                emin, mode, out.data_ptr(), stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("mode", [0, 1])
def test_noalloc_gradient_equals_workspace_gradient(mode):
    rng = np.random.default_rng(7 + mode)
    p32 = rng.normal(0.0, 0.4, 1249).astype(np.float32)
    # 300001 samples: 512 workgroups sweep several 128-sample chunks each;
    # then 5003 samples: 40 workgroups, ragged last chunk
    for n, seed in ((300001, 21), (5003, 22)):
        print(f"no-alloc gradient: mode={mode} n={n}", flush=True)
        E, M, eps = _samples(n, seed)
        a = _run("noalloc", p32, E, M, eps, mode)
        b = _run("ws", p32, E, M, eps, mode)
        assert np.all(np.isfinite(a)), (n, np.flatnonzero(~np.isfinite(a))[:8])
        np.testing.assert_array_equal(a, b)
        assert a[-1] > 0.5 * n  # the sample count: most samples are above emin
