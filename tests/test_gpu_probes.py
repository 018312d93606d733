"""The roof probes on the GPU: the copy kernel copies, and the FMA loop's
chains end where the arithmetic says (x_c = 1 + 0.001 (lane + c) plus
iters steps of 1e-6, summed over the 16 chains)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_copy_probe_copies():
    import torch

    from paper_2108_05602_amd import binding as B
    print("case: copy probe, 16 MiB and 48 bytes", flush=True)
    st = torch.cuda.current_stream().cuda_stream
    for n in (16 << 20, 48):
        src = torch.arange(n // 4, dtype=torch.int32, device="cuda:0")
        dst = torch.full((n // 4 + 64,), -1, dtype=torch.int32, device="cuda:0")
        B.fringe_probe_copy(src.data_ptr(), dst.data_ptr(), n, st)
        torch.cuda.synchronize()
        assert torch.equal(src, dst[: n // 4])
        assert torch.all(dst[n // 4:] == -1)   # nothing written past the n bytes


def test_fma_probe_values():
    import torch

    from paper_2108_05602_amd import binding as B
    print("case: FMA probe, 4 blocks x 1000 steps", flush=True)
    st = torch.cuda.current_stream().cuda_stream
    n_blocks, iters = 4, 1000
    out = torch.zeros(n_blocks * 256, dtype=torch.float32, device="cuda:0")
    flops = B.fringe_probe_fma(n_blocks, iters, out.data_ptr(), st)
    torch.cuda.synchronize()
    assert flops == 2.0 * 16 * iters * 256 * n_blocks
    lane = np.arange(256)
    expect = np.array([sum(1.0 + 0.001 * (l + c) + iters * 1e-6 for c in range(16)) for l in lane])
    got = out.cpu().numpy().reshape(n_blocks, 256)
    for b in range(n_blocks):
        np.testing.assert_allclose(got[b], expect, rtol=1e-3)
