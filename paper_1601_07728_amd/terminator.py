"""Learned continued-fraction terminator: dataset, training loop and spectrum assembly.

Orchestration only -- the recursion, the encoding, forward, backward, Adam, decoding and the
continued fraction run in the library's HIP kernels through the C ABI.  Torch holds device
arrays and draws the minibatch order (seeded); the host computes the training set's target
statistics that fix the loss weights and the starting point of the last layer.

Three ways to close the continued fraction after m = start + 32 Haydock steps (section 3.2's
recursion, eq. loss.fcn's spectrum):
  truncated  the m levels as they are (t = 0)
  sqrt       the constant-chain square-root terminator on the m levels
  mlp        the network, fed the window of 32 levels starting at `start`, extends the
             coefficients to start + 256 levels, then the square-root terminator closes them;
             sequences the network flags invalid fall back to the full-depth recursion when it
             is available, else to `sqrt`
A network is trained for one window start (the training sequences are cut to levels
start .. start + 255); the library ships one for start 0 (32 steps) and one for start 16
(48 steps).

Training recipe (measured on solver-generated SrTiO3-shaped data; see the design notes):
  * each output position j (224 a's, then 224 log b's, level n = 32 + j mod 224) is weighted by
    e^{-(n - 32)/tau} / var_j, var_j its variance over the training set: the outputs are put on
    one scale, and the first predicted levels, which set most of the spectrum at a 0.5 eV
    broadening, count most;
  * the hidden layers start He-normal, the last layer at zero weights and the mean target as
    bias, so the untrained network predicts the training set's mean tail;
  * Adam, learning rate 1e-3, minibatches of 64 in a seeded random order.
"""
from __future__ import annotations

import time

import numpy as np

from . import Bse, Mlp, spectrum

M_IN = 32
DEPTH = 256
N_OUT = DEPTH - M_IN
SIZES = (64, 256, 256, 256, 448)
# the full SrTiO3-shaped size of the dataset's systems: 8^3 k, 20^3 x, 96 bands
C2_SHAPE = dict(nk=(8, 8, 8), nx=(20, 20, 20), n_bands=96)
TAU = 16.0


def generate(seeds, n_steps: int = 512, precision: str = "bf16", shape=None, log=None):
    """Coefficients of the dipole recursions of each seeded system, three polarisations
    (x, y, z) per system, with u drawn on the device (synth.terminator_system_device).
    Returns dict with a, b [3 n_sys, n_steps], norm2, steps [3 n_sys], seeds [3 n_sys] (the
    system of each sequence) and seconds."""
    import synth
    shape = C2_SHAPE if shape is None else shape
    A, B, N2, SD, S = [], [], [], [], []
    t0 = time.perf_counter()
    for i, seed in enumerate(seeds):
        cr, u = synth.terminator_system_device(int(seed), n_steps=n_steps, **shape)
        h = Bse.from_crystal(cr, precision=precision, u=u)
        if precision != "fp64":
            del u                       # read only by create in the reduced-precision modes
        p0 = h.dipole_psi0(np.eye(3))
        a, b, n2, sd, _ = h.haydock(p0, n_steps)
        h.close()
        del p0
        A.append(a)
        B.append(b)
        N2.append(n2)
        SD.append(sd)
        S += [int(seed)] * 3
        if log is not None and (i + 1) % 16 == 0:
            log(f"terminator data: {i + 1} systems in {time.perf_counter() - t0:.1f} s")
    return {"a": np.concatenate(A), "b": np.concatenate(B), "norm2": np.concatenate(N2),
            "steps": np.concatenate(SD), "seeds": np.array(S), "seconds": time.perf_counter() - t0}


def host_targets(a, b):
    """The encoding's targets on the host (the same formula as the library's encode kernel),
    for the training set's statistics: (a_n - c)/s and log(b_n/s), n = 32..255."""
    c = a[:, 16:32].mean(axis=1, keepdims=True)
    s = b[:, 16:32].mean(axis=1, keepdims=True)
    return np.concatenate([(a[:, M_IN:DEPTH] - c) / s, np.log(b[:, M_IN:DEPTH] / s)], axis=1)


def loss_weights(t_train, tau: float = TAU):
    """Per-output weights e^{-(n - 32)/tau} / var_j, scaled to mean 1."""
    lev = np.concatenate([np.arange(N_OUT), np.arange(N_OUT)]).astype(np.float64)
    var = np.var(t_train, axis=0) + 1e-12
    w = np.exp(-lev / tau) / var
    return (w / w.mean()).astype(np.float32)


def init_params(t_train, rng):
    """He-normal hidden layers, zero biases; last layer zero weights with the mean target as
    bias.  Packed [W1, b1, ..., W4, b4], W stored [in][out]."""
    parts = []
    for li, (i, o) in enumerate(zip(SIZES[:-1], SIZES[1:])):
        last = li == len(SIZES) - 2
        parts.append(np.zeros(i * o) if last else rng.standard_normal(i * o) * np.sqrt(2.0 / i))
        parts.append(np.mean(t_train, axis=0) if last else np.zeros(o))
    return np.concatenate(parts).astype(np.float32)


def train(mlp: Mlp, x, t, epochs: int, batch: int, lr: float, seed: int = 0, log_every: int = 0):
    """Adam on minibatches of (x, t) (device float32 tensors) in a seeded random order.
    Returns the list of (epoch, mean minibatch loss) sampled every log_every epochs."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    n = x.shape[0]
    hist = []
    # a step without its loss returns with its work still queued on the network's stream,
    # reading the batch: the batch stays referenced (in_use) until the synchronisation before
    # the next step has retired that work, so torch cannot hand its memory to the next batch
    in_use = None
    for ep in range(epochs):
        perm = torch.randperm(n, device="cuda", generator=g)
        want = log_every > 0 and (ep % log_every == 0 or ep == epochs - 1)
        losses = []
        for s in range(0, n - batch + 1, batch):
            idx = perm[s:s + batch]
            xb = x.index_select(0, idx).contiguous()
            tb = t.index_select(0, idx).contiguous()
            torch.cuda.synchronize()
            in_use = (xb, tb)
            lv = mlp.train_step(xb, tb, lr, want_loss=want)
            if want:
                losses.append(lv)
        if want:
            hist.append((ep, float(np.mean(losses))))
    torch.cuda.synchronize()
    del in_use
    return hist


def fit(mlp: Mlp, a, b, epochs: int = 200, batch: int = 64, lr: float = 1e-3, seed: int = 0, tau: float = TAU,
        log_every: int = 0):
    """The training recipe above on coefficient sequences a, b [n, >= 256] (host FP64):
    encode on the device, weights and starting point from the targets' statistics, Adam.
    Returns the loss history."""
    import torch
    a = np.ascontiguousarray(a[:, :DEPTH])
    b = np.ascontiguousarray(b[:, :DEPTH])
    x, t = Mlp.encode(torch.from_numpy(a).to("cuda"), torch.from_numpy(b).to("cuda"))
    th = host_targets(a, b)
    mlp.set_params(init_params(th, np.random.default_rng(seed)))
    mlp.set_loss_weights(loss_weights(th, tau))
    return train(mlp, x, t, epochs=epochs, batch=batch, lr=lr, seed=seed, log_every=log_every)


def extend(mlp: Mlp, a, b, start: int = 0):
    """The network's extension of each sequence from its window of 32 levels starting at
    `start`: levels 0 .. start + 255, the first start + 32 as given.  Returns (a, b, valid)."""
    a = np.atleast_2d(a)
    b = np.atleast_2d(b)
    ae, be, valid = mlp.predict(np.ascontiguousarray(a[:, start:start + M_IN]),
                                np.ascontiguousarray(b[:, start:start + M_IN]))
    if start == 0:
        return ae, be, valid
    return np.concatenate([a[:, :start], ae], axis=1), np.concatenate([b[:, :start], be], axis=1), valid


def _per_omega(fn, omegas):
    """Apply fn(rows, omega) to the groups of rows sharing one energy grid; stack the results."""
    out = [None] * len(omegas)
    keys = {}
    for i, om in enumerate(omegas):
        keys.setdefault((len(om), float(om[0]), float(om[-1])), []).append(i)
    for rows in keys.values():
        sig = fn(np.array(rows), omegas[rows[0]])
        for j, r in enumerate(rows):
            out[r] = sig[j]
    return np.array(out)


def terminated_spectra(mlp: Mlp, a, b, norm2, omega, gamma, a_full=None, b_full=None, n_full=None,
                       start: int = 0):
    """Spectra of each sequence closed three ways after start + 32 steps (see the module
    docstring).  a, b [n, >= start + 32] host arrays; omega: one grid, or a list of
    per-sequence grids.  Returns dict name -> sigma [n, n_omega] and the validity mask."""
    a = np.atleast_2d(a)
    b = np.atleast_2d(b)
    n = a.shape[0]
    omegas = omega if isinstance(omega, (list, tuple)) else [omega] * n
    norm2 = np.atleast_1d(norm2)
    m = start + M_IN
    mm = np.full(n, m, dtype=np.int32)
    out = {
        "truncated": _per_omega(lambda r, om: spectrum(a[r, :m], b[r, :m], norm2[r], om, gamma, "none",
                                                       n_used=mm[r]), omegas),
        "sqrt": _per_omega(lambda r, om: spectrum(a[r, :m], b[r, :m], norm2[r], om, gamma, "sqrt",
                                                  n_used=mm[r]), omegas),
    }
    ae, be, valid = extend(mlp, a, b, start)
    sig = _per_omega(lambda r, om: spectrum(ae[r], be[r], norm2[r], om, gamma, "sqrt"), omegas)
    if not valid.all():
        bad = np.nonzero(~valid)[0]
        for i in bad:
            if a_full is not None:
                sig[i] = spectrum(a_full[i:i + 1], b_full[i:i + 1], norm2[i:i + 1], omegas[i], gamma, "none",
                                  n_used=None if n_full is None else n_full[i:i + 1])[0]
            else:
                sig[i] = out["sqrt"][i]
    out["mlp"] = sig
    return out, valid


def reference_spectra(a, b, norm2, omega, gamma, n_used=None):
    """Full-depth spectra (no terminator) on one or per-sequence grids."""
    a = np.atleast_2d(a)
    n = a.shape[0]
    omegas = omega if isinstance(omega, (list, tuple)) else [omega] * n
    used = None if n_used is None else np.atleast_1d(n_used)
    return _per_omega(lambda r, om: spectrum(a[r], b[r], np.atleast_1d(norm2)[r], om, gamma,
                                             n_used=None if used is None else used[r]), omegas)


def l1(sig, ref):
    """Per-row relative L1 distance on the uniform grid."""
    return np.sum(np.abs(sig - ref), axis=-1) / np.sum(np.abs(ref), axis=-1)
