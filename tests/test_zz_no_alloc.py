"""The allocation-free prediction entry point (ocean_mlp_predict_noalloc) against
ocean_mlp_predict, through the C ABI, on two calls in a row (the second smaller), on the
default stream and on a stream of the caller's."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _chains(rng, n, stride):
    """Coefficient sequences shaped like Haydock output: a near a band centre, b > 0."""
    a = 0.6 + 0.2 * rng.standard_normal((n, stride))
    b = 0.2 + 0.05 * rng.uniform(0.0, 1.0, (n, stride))
    return a, b


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
def test_noalloc_predict_equals_predict(precision):
    import torch
    import paper_1601_07728_amd as ob
    m = ob.Mlp(precision)
    rng = np.random.default_rng(31)
    m.set_params((0.05 * rng.standard_normal(m.n_params)).astype(np.float32))
    side = torch.cuda.Stream()
    for n, stride, stream in ((300, 40, None), (37, 32, side)):
        print(f"no-alloc predict: {precision}, n_seq {n}, stride {stride}, "
              f"{'caller stream' if stream else 'default stream'}", flush=True)
        a, b = _chains(rng, n, stride)
        ae, be, valid = m.predict(a, b)
        a_d = torch.from_numpy(a).cuda()
        b_d = torch.from_numpy(b).cuda()
        ae_d = torch.full((n, 256), float("nan"), dtype=torch.float64, device="cuda")
        be_d = torch.full((n, 256), float("nan"), dtype=torch.float64, device="cuda")
        v_d = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        m.predict_noalloc(a_d, b_d, ae_d, be_d, v_d, stream=stream)
        torch.cuda.synchronize()
        assert np.array_equal(ae_d.cpu().numpy(), ae)
        assert np.array_equal(be_d.cpu().numpy(), be)
        assert np.array_equal(v_d.cpu().numpy().astype(bool), valid)
        assert valid.all()
        assert np.array_equal(ae[:, :32], a[:, :32]) and np.array_equal(be[:, :32], b[:, :32])
    m.close()


def test_noalloc_predict_rejects_more_sequences_than_the_scratch_holds():
    import torch
    import paper_1601_07728_amd as ob
    m = ob.Mlp("bf16")
    n = ob.MLP_NOALLOC_MAX_SEQ + 1
    a = torch.ones((n, 32), dtype=torch.float64, device="cuda")
    ae = torch.zeros((n, 256), dtype=torch.float64, device="cuda")
    v = torch.zeros((n,), dtype=torch.int32, device="cuda")
    with pytest.raises(ob.OceanError) as e:
        m.predict_noalloc(a, a, ae, ae.clone(), v)
    assert e.value.code == ob.ERR_INVALID_ARG and "exceeds" in str(e.value)
    m.close()
