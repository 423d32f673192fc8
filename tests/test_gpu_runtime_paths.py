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
