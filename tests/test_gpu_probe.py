"""The gather probe (include/ecc_probe.h) reads what it is given: with a
buffer of ones every thread's sum is 4 x iters, for both access patterns and
buffer sizes from 1 KiB up; its argument checks refuse bad sizes."""
import numpy as np
import pytest

from paper_1806_02637_amd import binding as B

pytestmark = pytest.mark.gpu


def test_probe_reads_every_load():
    import torch

    print("case: gather probe", flush=True)
    stream = torch.cuda.current_stream().cuda_stream
    for nbytes in (1 << 10, 1 << 21, 1 << 27):
        buf = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        for pattern in (0, 1):
            for iters, blocks in ((4, 1), (64, 37)):
                out = torch.full((blocks * 256,), -1.0, dtype=torch.float32, device="cuda")
                B.ecc_probe_gather(buf.data_ptr(), nbytes, pattern, iters, blocks, out.data_ptr(), stream)
                torch.cuda.synchronize()
                assert np.all(out.cpu().numpy() == 4.0 * iters), (nbytes, pattern, iters)
    out = torch.empty(256, dtype=torch.float32, device="cuda")
    buf = torch.ones(1024, dtype=torch.float32, device="cuda")
    for args in ((3000, 0, 4, 1), (4096, 2, 4, 1), (4096, 0, 6, 1), (4096, 0, 4, 0)):
        with pytest.raises(B.EccError) as ei:
            B.ecc_probe_gather(buf.data_ptr(), *args, out.data_ptr(), stream)
        assert ei.value.status == B.ECC_E_ARG
