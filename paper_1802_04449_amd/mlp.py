"""Training driver of the learned root-solve guess (ktmi_mlp_* in include/ktmi.h).

The network (4 -> 32 -> 32 -> 1, tanh) maps features of K = (E, K^i) to a start
inside the root bracket [lo, E] of the per-cell root solve.  Training samples
(E, M = |K^i|, e) come from states of the hydro step itself (ktmi_harvest);
forward, backward and Adam run in the library's kernels.  This module only
prepares the sample arrays (filter, shuffle: host side), initialises the
parameters and sequences the calls.
"""
from __future__ import annotations

import math

import numpy as np

from . import (KTMI_MLP_FP32, ktmi_mlp_adam, ktmi_mlp_forward, ktmi_mlp_grad,
               ktmi_mlp_grad_workspace_bytes, ktmi_mlp_nparam)

NH = 32
# flat parameter layout: W1[32][4], b1[32], W2[32][32], b2[32], w3[32], b3
OW1, OB1, OW2, OB2, OW3, OB3 = 0, 128, 160, 1184, 1216, 1248


def init_params(seed: int = 0) -> np.ndarray:
    """Glorot-uniform weights, zero biases (float32, host)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(ktmi_mlp_nparam(), dtype=np.float32)

    def glorot(fan_in, fan_out, size):
        b = math.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-b, b, size).astype(np.float32)

    p[OW1:OB1] = glorot(4, NH, NH * 4)
    p[OW2:OB2] = glorot(NH, NH, NH * NH)
    p[OW3:OB3] = glorot(NH, 1, NH)
    return p


def samples_from_states(states, emin: float, seed: int = 0):
    """Concatenates harvested (E, M, e) device triples and shuffles them (host);
    returns float64 host arrays.  Kept: E >= emin and e >= emin.  A cell whose
    root fell below the cutoff reports e = 0, a target outside the bracket the
    network's output lives in; such cells are left out."""
    E, M, e = [], [], []
    for (a, b, c) in states:
        a, b, c = (x.cpu().numpy() for x in (a, b, c))
        keep = np.isfinite(a) & np.isfinite(b) & (a >= emin) & (c >= emin)
        E.append(a[keep])
        M.append(b[keep])
        e.append(c[keep])
    E, M, e = np.concatenate(E), np.concatenate(M), np.concatenate(e)
    perm = np.random.default_rng(seed).permutation(E.size)
    return E[perm], M[perm], e[perm]


class Trainer:
    """Adam on device-resident samples; minibatches are contiguous slices of the
    shuffled arrays, taken in order and wrapping around."""

    def __init__(self, E, M, eps, device="cuda", stream=None, mode=KTMI_MLP_FP32, seed=0,
                 emin=1e-7):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).to(self.device)
        self.E, self.M, self.eps = dev(E), dev(M), dev(eps)
        self.n = int(self.E.numel())
        self.mode = mode
        self.emin = emin
        n = ktmi_mlp_nparam()
        self.params = torch.as_tensor(init_params(seed)).to(self.device)
        self.m = torch.zeros(n, dtype=torch.float32, device=self.device)
        self.v = torch.zeros(n, dtype=torch.float32, device=self.device)
        self.out = torch.zeros(n + 2, dtype=torch.float32, device=self.device)
        self.t = 0
        self.pos = 0
        self._ws = None
        self._ws_n = 0

    def _workspace(self, n):
        if self._ws is None or self._ws_n < n:
            nb = ktmi_mlp_grad_workspace_bytes(n)
            self._ws = self.torch.empty(nb // 4 + 64, dtype=self.torch.float32, device=self.device)
            self._ws_n = n
        return self._ws

    def grad(self, off=0, count=None):
        """Gradient, mean loss and count over samples [off, off + count)."""
        count = self.n - off if count is None else count
        ws = self._workspace(count)
        s = self.stream.cuda_stream
        ktmi_mlp_grad(self.params.data_ptr(), count, self.E.data_ptr() + 8 * off,
                      self.M.data_ptr() + 8 * off, self.eps.data_ptr() + 8 * off, self.emin,
                      self.mode, self.out.data_ptr(), ws.data_ptr(),
                      ktmi_mlp_grad_workspace_bytes(count), s)
        return self.out

    def step(self, batch, lr=3e-3, b1=0.9, b2=0.999, epsilon=1e-8):
        if self.pos + batch > self.n:
            self.pos = 0
        self.grad(self.pos, min(batch, self.n))
        self.pos += batch
        self.t += 1
        ktmi_mlp_adam(self.params.data_ptr(), self.out.data_ptr(), self.m.data_ptr(),
                      self.v.data_ptr(), self.t, lr, b1, b2, epsilon, self.stream.cuda_stream)

    def train(self, steps, batch=8192, lr=3e-3, lr_final=3e-4, log_every=0):
        """Adam with an exponential learning-rate decay from lr to lr_final;
        returns [(t, mean loss of the batch)] every log_every steps."""
        hist = []
        for k in range(steps):
            a = k / max(steps - 1, 1)
            self.step(batch, lr=lr * (lr_final / lr) ** a)
            if log_every and (k + 1) % log_every == 0:
                self.stream.synchronize()
                hist.append((self.t, float(self.out[-2].item())))
        self.stream.synchronize()
        return hist

    def loss(self):
        """Mean loss over all samples."""
        self.grad(0, self.n)
        self.stream.synchronize()
        return float(self.out[-2].item())

    def forward(self, E, M, emin=None):
        t = self.torch
        E = t.as_tensor(E, dtype=t.float64, device=self.device).contiguous()
        M = t.as_tensor(M, dtype=t.float64, device=self.device).contiguous()
        g = t.empty_like(E)
        ktmi_mlp_forward(self.params.data_ptr(), E.numel(), E.data_ptr(), M.data_ptr(),
                         self.emin if emin is None else emin, g.data_ptr(), self.mode,
                         self.stream.cuda_stream)
        return g
