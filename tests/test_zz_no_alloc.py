"""The allocation-free misfit residual (rtm_misfit_residual_chunks_noalloc) against the entry point
that takes the caller's partial-sum buffer: the same residual and the same FP64 misfit bits, on two
calls in a row, the second with a smaller input (fewer samples and chunks), so nothing from the first
call's use of the library's scratch may leak into the second."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_noalloc_residual_matches_buffered_entry_point():
    import torch

    from paper_1603_03971_amd import _abi

    st = torch.cuda.current_stream()
    rng = np.random.default_rng(77)
    for n, nchunks in ((3_000_017, 4096), (50_011, 37), (1, 1)):
        d = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).cuda()
        obs = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).cuda()
        ra, rb = torch.empty_like(d), torch.full_like(d, float("nan"))
        ma = torch.zeros(1, dtype=torch.float64, device="cuda")
        mb = torch.zeros(1, dtype=torch.float64, device="cuda")
        partials = torch.empty(nchunks, dtype=torch.float64, device="cuda")
        _abi.rtm_misfit_residual_chunks(d, obs, ra, n, partials, nchunks, ma, st)
        before = torch.cuda.memory_allocated()
        _abi.rtm_misfit_residual_chunks_noalloc(d, obs, rb, n, nchunks, mb, st)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        assert torch.equal(ra, rb)
        assert ma.item() == mb.item(), (n, ma.item(), mb.item())
        r32 = d.cpu().numpy() - obs.cpu().numpy()           # the residual is formed in FP32
        assert np.array_equal(rb.cpu().numpy(), r32)
        r64 = r32.astype(np.float64)
        ref = 0.5 * float(np.sum(r64 * r64))
        assert abs(mb.item() - ref) <= 1e-12 * ref
        print(f"n {n} nchunks {nchunks}: misfit {mb.item():.17g} (FP64 reference {ref:.17g})", flush=True)


def test_noalloc_rejects_too_many_chunks():
    import torch

    from paper_1603_03971_amd import _abi

    d = torch.zeros(10, device="cuda")
    m = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(_abi.RTMError) as e:
        _abi.rtm_misfit_residual_chunks_noalloc(d, d, d, 10, 4097, m)
    assert e.value.status == _abi.RTM_EINVAL
    with pytest.raises(_abi.RTMError) as e:
        _abi.rtm_misfit_residual_chunks_noalloc(d, d, d, 10, 0, m)
    assert e.value.status == _abi.RTM_EINVAL
