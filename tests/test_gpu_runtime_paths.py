"""Runtime paths forced from the host: the device-memory cap (OCEAN_MAX_DEVICE_BYTES) turns
an allocation past it into OUT_OF_MEMORY, at create and at the recursion's first use of its
buffers, and leaves the handle usable once lifted; the eager step loop (OCEAN_NO_GRAPH)
gives the same coefficients as the replayed graph, bit for bit, alone and batched; per-kernel
timing reports every kernel of the step and changes no result."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_device_memory_cap(monkeypatch):
    import paper_1601_07728_amd as ob
    cr = synth.small_l_edge(seed=81, nk=(2, 2, 2), nx=(6, 6, 5), n_bands=14)
    monkeypatch.setenv("OCEAN_MAX_DEVICE_BYTES", "4096")
    with pytest.raises(ob.OceanError) as e:
        ob.Bse.from_crystal(cr, precision="fp64")
    assert e.value.code == ob.ERR_OUT_OF_MEMORY
    monkeypatch.delenv("OCEAN_MAX_DEVICE_BYTES")
    h = ob.Bse.from_crystal(cr, precision="fp64")
    held = h.device_bytes
    p0 = h.dipole_psi0(np.eye(3))
    monkeypatch.setenv("OCEAN_MAX_DEVICE_BYTES", str(held + 1024))
    with pytest.raises(ob.OceanError) as e:
        h.haydock(p0, 20)
    assert e.value.code == ob.ERR_OUT_OF_MEMORY
    monkeypatch.delenv("OCEAN_MAX_DEVICE_BYTES")
    a, b, n2, sd, rc = h.haydock(p0, 20)
    assert rc == ob.OK and np.all(sd == 20)
    h.close()


def test_eager_steps_equal_graph_replay(monkeypatch):
    import paper_1601_07728_amd as ob
    crs = [synth.small_l_edge(seed=82 + s, nk=(2, 2, 2), nx=(5, 6, 5), n_bands=11 + 4 * s) for s in range(3)]
    runs = {}
    for mode in ("graph", "eager"):
        if mode == "eager":
            monkeypatch.setenv("OCEAN_NO_GRAPH", "1")
        hs = [ob.Bse.from_crystal(cr, precision="fp64") for cr in crs]
        p0 = [h.dipole_psi0(np.eye(3)) for h in hs]
        single = hs[0].haydock(p0[0], 30)
        batch, rc = ob.haydock_batch(hs, p0, 30)
        runs[mode] = (single, batch)
        for h in hs:
            h.close()
    (sg, bg), (se, be) = runs["graph"], runs["eager"]
    assert np.array_equal(sg[0], se[0]) and np.array_equal(sg[1], se[1])
    for (ag, bgg, ng, sdg), (ae, bee, ne, sde) in zip(bg, be):
        assert np.array_equal(ag, ae) and np.array_equal(bgg, bee) and np.array_equal(sdg, sde)


def test_profiling_times_every_kernel_and_changes_nothing():
    """With per-kernel timing on, the recursion runs its kernels eagerly between HIP events:
    the coefficients equal the graph-replayed ones bit for bit, and every kernel of the step
    is reported once per step with a positive time."""
    import paper_1601_07728_amd as ob
    cr = synth.small_l_edge(seed=85, nk=(2, 2, 2), nx=(6, 5, 6), n_bands=15)
    h = ob.Bse.from_crystal(cr, precision="fp64")
    p0 = h.dipole_psi0(np.eye(3))
    a, b, n2, sd, rc = h.haydock(p0, 12)
    h.set_profiling(True)
    ap, bp, n2p, sdp, rcp = h.haydock(p0, 12)
    kt = h.kernel_times()
    h.set_profiling(False)
    h.close()
    assert np.array_equal(a, ap) and np.array_equal(b, bp) and np.array_equal(n2, n2p)
    for name in ("proj_fwd", "proj_bwd", "fft_w", "combine", "local_in", "local_mat", "lz_update",
                 "lz_finalize", "lz_scale"):
        assert name in kt, (name, sorted(kt))
        ms, count = kt[name]
        assert ms > 0.0 and count == 12, (name, ms, count)


@pytest.mark.parametrize("bad", ["0 0 0 0 8", "3 2048 16 0 8", "1 777 16 0 8", "1 2048 0 0 8", "2 1024 48 0 8",
                                 "1 2048 128 0 8", "1 2048 16 5 8", "1 2048 16 0 3", "1 2048 16 0 0", "1 2048 16 0"])
def test_corrupt_autotune_cache_line_is_tuned_again(monkeypatch, tmp_path, bad):
    """A cached tile choice that the tuner could not have made (zero or odd knobs, lines past
    the transform's 160 KiB LDS budget) is ignored: the shape is tuned again, the new choice is
    valid and appended, and H*v is unchanged."""
    import torch
    import paper_1601_07728_amd as ob
    cr = synth.small_l_edge(seed=84, nk=(2, 2, 2), nx=(6, 5, 6), n_bands=13)
    h = ob.Bse.from_crystal(cr, precision="fp64")
    p0 = h.dipole_psi0(np.eye(3))
    y0 = h.apply(p0).cpu().numpy()
    key = f"ocean-tune-v5 nk=2,2,2 nx=6,5,6 nb=13 nc=6 nmu=5 prec=0 cols={3 * cr.n_core}"
    cache = tmp_path / "tune.txt"
    cache.write_text(f"{key}|{bad}\n")
    monkeypatch.setenv("OCEAN_AUTOTUNE_CACHE", str(cache))
    h.autotune(3, reps=2)
    t = h.tuning
    ms, bt, fl, ft, bw = t["fwd_ms"], t["bwd_blocks"], t["fft_lines"], t["fwd_tiles"], t["bwd_waves"]
    assert ms in (1, 2) and bt in (1024, 2048, 4096, 8192) and fl in (4, 8, 16, 32, 64) and ft in (0, 4, 8, 16, 32)
    assert bw in (2, 4, 8)
    lines = cache.read_text().splitlines()
    assert len(lines) == 2 and lines[1] == f"{key}|{ms} {bt} {fl} {ft} {bw}"
    y1 = h.apply(p0).cpu().numpy()
    assert np.abs(y1 - y0).max() <= 1e-13 * np.abs(y0).max()
    # a valid line is reused as it stands
    h2 = ob.Bse.from_crystal(cr, precision="fp64")
    cache.write_text(f"{key}|2 4096 8 16 4\n")
    h2.autotune(3, reps=2)
    assert h2.tuning == {"fwd_ms": 2, "bwd_blocks": 4096, "fft_lines": 8, "fwd_tiles": 16, "bwd_waves": 4}
    torch.cuda.synchronize()
    h.close()
    h2.close()
