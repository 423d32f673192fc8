"""Build the learned terminator's dataset and train the shipped network.

  python -m paper_1601_07728_amd.train_terminator generate FIRST COUNT OUT.npz
      the dipole recursions (512 steps, x, y, z polarisations) of terminator systems
      FIRST .. FIRST + COUNT - 1 at the full SrTiO3-shaped size (8^3 k, 20^3 x, 96 bands,
      eps ~ U[2, 10], band width ~ U[20, 60] eV), on the GPU with BF16 projections
  python -m paper_1601_07728_amd.train_terminator train START OUT_MODEL.npz DATA.npz [DATA.npz ...]
      train the network with the library's kernels (terminator.fit) on every sequence of the
      data files whose system seed is a training seed, cut to levels START .. START + 255 (the
      network then extends the recursion from START + 32 steps), and write its parameters

Training systems are seeds 1..TRAIN_SYSTEMS (3 polarisations each, 3840 sequences); seeds
HELD_OUT are never trained on and judge the network.  The model file holds the FP32
parameters, the window start and the recipe; MODEL_FILES names the shipped networks by window
start.
"""
from __future__ import annotations

import sys
import time

import numpy as np

TRAIN_SYSTEMS = 1280
HELD_OUT = range(1281, 1367)       # 86 systems, 258 sequences
MODEL_FILE = "terminator_srtio3_l23.npz"            # window start 0: closes 32-step recursions
MODEL_FILES = {0: MODEL_FILE, 16: "terminator_srtio3_l23_w16.npz"}   # by window start


def _log(msg):
    print(f"[train_terminator] {msg}", flush=True)


def generate(first: int, count: int, out: str):
    from . import terminator as term
    d = term.generate(range(first, first + count), log=_log)
    np.savez_compressed(out, a=d["a"], b=d["b"], norm2=d["norm2"], steps=d["steps"], seeds=d["seeds"],
                        seconds=d["seconds"])
    _log(f"{count} systems ({3 * count} sequences) in {d['seconds']:.1f} s -> {out}")


def train(out: str, files, epochs: int = 200, start: int = 0):
    from . import Mlp
    from . import terminator as term
    parts = [np.load(f) for f in files]
    a = np.concatenate([p["a"] for p in parts])
    b = np.concatenate([p["b"] for p in parts])
    seeds = np.concatenate([p["seeds"] for p in parts])
    steps = np.concatenate([p["steps"] for p in parts])
    keep = (seeds >= 1) & (seeds <= TRAIN_SYSTEMS) & (steps >= start + term.DEPTH)
    a, b = a[keep][:, start:start + term.DEPTH], b[keep][:, start:start + term.DEPTH]
    _log(f"{a.shape[0]} training sequences from {len(np.unique(seeds[keep]))} systems")
    m = Mlp("bf16")
    t0 = time.perf_counter()
    hist = term.fit(m, a, b, epochs=epochs, log_every=max(1, epochs // 10))
    dt = time.perf_counter() - t0
    _log(f"trained {epochs} epochs in {dt:.1f} s; loss {hist}")
    np.savez(out, params=m.get_params(), start=start, tau=term.TAU, epochs=epochs, batch=64, lr=1e-3,
             n_sequences=a.shape[0], train_systems=TRAIN_SYSTEMS, train_seconds=dt,
             loss_history=np.array(hist))
    m.close()


if __name__ == "__main__":
    cmd = sys.argv[1]
    if cmd == "generate":
        generate(int(sys.argv[2]), int(sys.argv[3]), sys.argv[4])
    elif cmd == "train":
        train(sys.argv[3], sys.argv[4:], start=int(sys.argv[2]))
    else:
        raise SystemExit(__doc__)
