"""seis_combine_noalloc (the superposition for callers that cannot allocate
device memory) against seis_combine, through the C ABI: identical records on
two calls in a row, the second with a smaller input, and a clear refusal of an
event list larger than its static device memory."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B(gpu):
    from paper_1705_04874_amd import binding
    return binding


def run_both(B, n_src, n_rec, nt_in, n_ev, nt_out, dt_in, dt_out, seed):
    import torch
    rng = np.random.default_rng(seed)
    tr = torch.from_numpy(rng.standard_normal((n_src, 4, n_rec, nt_in)).astype(np.float32)).cuda()
    t0 = [dt_in, 0.5 * dt_in, 0.5 * dt_in, 0.5 * dt_in]
    src = rng.integers(0, n_src, n_ev).astype(np.int32)
    amp = rng.lognormal(0.0, 1.0, n_ev)
    to = rng.uniform(-0.1 * nt_out * dt_out, 1.1 * nt_out * dt_out, n_ev)
    ref = B.seis_combine(tr, t0, src, amp, to, nt_out, dt_in, dt_out)
    out = torch.full((4, n_rec, nt_out), np.nan, dtype=torch.float32, device="cuda")
    got = B.seis_combine(tr, t0, src, amp, to, nt_out, dt_in, dt_out, out=out, noalloc=True)
    assert got.data_ptr() == out.data_ptr()
    return got.cpu().numpy(), ref.cpu().numpy()


def test_noalloc_equals_seis_combine_on_two_calls_in_a_row(B):
    # first call: two record segments, long input rows (two staging chunks)
    got, ref = run_both(B, n_src=6, n_rec=33, nt_in=5000, n_ev=120, nt_out=20000, dt_in=0.8e-3, dt_out=1e-3, seed=1)
    np.testing.assert_array_equal(got, ref)
    assert np.abs(ref).max() > 0
    # second call, smaller: the static lists of the first call must not leak into it
    got, ref = run_both(B, n_src=2, n_rec=5, nt_in=300, n_ev=7, nt_out=900, dt_in=1e-3, dt_out=0.7e-3, seed=2)
    np.testing.assert_array_equal(got, ref)
    assert np.abs(ref).max() > 0


def test_noalloc_refuses_event_lists_beyond_its_memory(B):
    import torch
    cap = int(B._L.seis_combine_noalloc_max_bytes())
    assert cap == 4 << 20
    n_ev = cap // 16 + 1000                     # more event entries than fit in one segment's list
    tr = torch.zeros((2, 4, 3, 50), device="cuda")
    out = torch.zeros((4, 3, 100), device="cuda")
    with pytest.raises(B.PstdError) as e:
        B.seis_combine(tr, [0.0] * 4, np.zeros(n_ev, np.int32), np.ones(n_ev), np.zeros(n_ev), 100, 1e-3, 1e-3,
                       out=out, noalloc=True)
    assert e.value.code == B.PSTD_EINVAL and "static device memory" in str(e.value)
    assert not out.any()
