"""vsh_generate_into_static (the entry point for callers that cannot allocate)
against vsh_generate_into on the same requests, through the C ABI: two calls
in a row, the second with a smaller request, so the second reuses the
library's static workspace with the first call's contents still in it.
Per-event summaries must be bitwise equal (the same kernels on the same
inputs); histograms equal up to the order of their FP64 atomic sums."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2403_08692_amd as P

    c = P.Context()
    yield c
    c.close()


def _buffers(torch, dev, n, P):
    return (torch.zeros(P.HIST_DOUBLES, dtype=torch.float64, device=dev),
            torch.full((P.NSUM_D, n), -7.0, dtype=torch.float64, device=dev),
            torch.full((P.NSUM_I, n), -7, dtype=torch.int32, device=dev),
            torch.zeros(n, dtype=torch.int64, device=dev))


def test_static_workspace_matches_caller_workspace(ctx):
    import torch

    import paper_2403_08692_amd as P
    from paper_2403_08692_amd._native import make_request

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    cases = [(9000, 91.2, 1.0, 64, 21), (2500, 200.0, 0.5, 128, 22)]  # the second call is smaller
    for n, ecm, tc, cap, seed in cases:
        req, keep = make_request(n, seed, 0, ecm, tc, cap, P.VSH_FORM_PLAIN)
        ws_bytes = ctx.workspace_size(req)
        assert ws_bytes <= P.STATIC_SCRATCH_BYTES
        print(f"case static workspace n={n} ecm={ecm} cap={cap} ws={ws_bytes}", flush=True)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
        a = _buffers(torch, dev, n, P)
        b = _buffers(torch, dev, n, P)
        ctx.generate_into(req, stream.cuda_stream, ws.data_ptr(), ws_bytes, *[t.data_ptr() for t in a])
        ctx.generate_into_static(req, stream.cuda_stream, *[t.data_ptr() for t in b])
        torch.cuda.synchronize()
        ha, sda, sia, hsa = [t.cpu().numpy() for t in a]
        hb, sdb, sib, hsb = [t.cpu().numpy() for t in b]
        np.testing.assert_array_equal(sib, sia)
        np.testing.assert_array_equal(hsb, hsa)
        np.testing.assert_array_equal(sdb, sda)
        np.testing.assert_allclose(hb, ha, rtol=1e-11, atol=1e-9)
        assert (sia[1] == 1).mean() > 0.99 and sia[3].sum() > n


def test_static_workspace_refuses_what_it_cannot_hold(ctx):
    import torch

    import paper_2403_08692_amd as P
    from paper_2403_08692_amd._native import make_request

    dev = torch.device("cuda:0")
    hist = torch.zeros(P.HIST_DOUBLES, dtype=torch.float64, device=dev)
    big, keep = make_request(200_000, 1, 0, 91.2, 1.0, 64, P.VSH_FORM_PLAIN)
    assert ctx.workspace_size(big) > P.STATIC_SCRATCH_BYTES
    with pytest.raises(P.VshError) as ei:
        ctx.generate_into_static(big, 0, hist.data_ptr())
    assert ei.value.code == -2 and "static workspace" in str(ei.value)
    pers, keep = make_request(1000, 1, 0, 91.2, 1.0, 64, P.VSH_FORM_PERSISTENT)
    with pytest.raises(P.VshError) as ei:
        ctx.generate_into_static(pers, 0, hist.data_ptr())
    assert ei.value.code == -1
    torch.cuda.synchronize()
    assert float(hist.abs().sum().cpu()) == 0.0  # refused calls launch nothing
