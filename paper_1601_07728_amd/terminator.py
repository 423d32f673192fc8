"""Learned continued-fraction terminator: training loop and spectrum assembly.

Orchestration only -- every arithmetic step (encoding, forward, backward, Adam, decoding,
continued fraction) runs in the library's HIP kernels through the C ABI.  Torch holds
device arrays and draws the minibatch order (seeded).

Three ways to close the continued fraction after m = 32 Haydock steps (section 3.2's
recursion, eq. loss.fcn's spectrum):
  truncated  the 32 levels as they are (t = 0)
  sqrt       the constant-chain square-root terminator on the 32 levels
  mlp        the network extends the coefficients to 256 levels, then the square-root
             terminator closes them; sequences the network flags invalid fall back to the
             full-depth recursion when it is available, else to `sqrt`
"""
from __future__ import annotations

import numpy as np

from . import Mlp, spectrum

M_IN = 32
DEPTH = 256


def train(mlp: Mlp, x, t, epochs: int, batch: int, lr: float, seed: int = 0, log_every: int = 0):
    """Adam on minibatches of (x, t) (device float32 tensors) in a seeded random order.
    Returns the list of (epoch, mean minibatch loss) sampled every log_every epochs."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    n = x.shape[0]
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, device="cuda", generator=g)
        want = log_every > 0 and (ep % log_every == 0 or ep == epochs - 1)
        losses = []
        for s in range(0, n - batch + 1, batch):
            idx = perm[s:s + batch]
            xb = x.index_select(0, idx).contiguous()
            tb = t.index_select(0, idx).contiguous()
            torch.cuda.synchronize()
            lv = mlp.train_step(xb, tb, lr, want_loss=want)
            if want:
                losses.append(lv)
        if want:
            hist.append((ep, float(np.mean(losses))))
    torch.cuda.synchronize()
    return hist


def terminated_spectra(mlp: Mlp, a, b, norm2, omega, gamma, a_full=None, b_full=None, n_full=None):
    """Spectra of each sequence closed three ways (see the module docstring).
    a, b [n, >=32] host arrays; returns dict name -> sigma [n, n_omega] and the validity mask."""
    a = np.atleast_2d(a)
    b = np.atleast_2d(b)
    n = a.shape[0]
    m32 = np.full(n, M_IN, dtype=np.int32)
    out = {
        "truncated": spectrum(a[:, :M_IN], b[:, :M_IN], norm2, omega, gamma, "none", n_used=m32),
        "sqrt": spectrum(a[:, :M_IN], b[:, :M_IN], norm2, omega, gamma, "sqrt", n_used=m32),
    }
    ae, be, valid = mlp.predict(a[:, :M_IN], b[:, :M_IN])
    sig = spectrum(ae, be, norm2, omega, gamma, "sqrt")
    if not valid.all():
        bad = np.nonzero(~valid)[0]
        if a_full is not None:
            sig[bad] = spectrum(a_full[bad], b_full[bad], norm2[bad], omega, gamma, "none",
                                n_used=None if n_full is None else n_full[bad])
        else:
            sig[bad] = out["sqrt"][bad]
    out["mlp"] = sig
    return out, valid


def l1(sig, ref):
    """Per-row relative L1 distance on the uniform grid."""
    return np.sum(np.abs(sig - ref), axis=-1) / np.sum(np.abs(ref), axis=-1)
