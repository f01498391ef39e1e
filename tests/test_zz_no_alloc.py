"""The allocation-free cost entry point (ecc_cost_noalloc), called through
the C ABI, against ecc_cost with a caller workspace.  Both run the same
kernels in the same order, so costs and per-pair terms must agree bit for
bit.  Two calls in a row, the second on a smaller input (fewer views, fewer
hypotheses, so the static scratch still holds the first call's larger
contents), then the first input again, and an evaluation too large for the
static scratch, which must be refused with a clear error."""
import math

import numpy as np
import pytest

from paper_1806_02637_amd import binding as B
from paper_1806_02637_amd import inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def eng():
    import torch

    from paper_1806_02637_amd import engine

    assert torch.cuda.is_available()
    e = engine.Engine(0)
    yield e
    e.close()


def _scan(eng, n_views, seed):
    g = inputs.ScanGeometry(n_views, 128, 128, 2.4)
    scan = eng.load_scan(g.projection_matrices(), g.intrinsics(), inputs.project(g, inputs.random_phantom(seed, 10)))
    scan.build_sinograms(180, 181, 0.5, "f32")
    return g, scan


def _both(eng, scan, theta, params):
    """(cost, pairs) of ecc_cost with its own workspace and of
    ecc_cost_noalloc, on the same stream."""
    import torch

    dev = eng.device
    th = torch.as_tensor(theta, dtype=torch.float64, device=dev).contiguous()
    Bn = th.shape[0]
    stream = torch.cuda.current_stream(dev).cuda_stream
    out = []
    for noalloc in (False, True):
        cost = torch.full((Bn,), math.nan, dtype=torch.float64, device=dev)
        pairs = torch.full((Bn, scan.n_pairs), math.nan, dtype=torch.float32, device=dev)
        if noalloc:
            B.ecc_cost_noalloc(eng.ctx, scan.id, Bn, th.data_ptr(), params, cost.data_ptr(), pairs.data_ptr(), stream)
        else:
            ws = scan.workspace(Bn, False)
            B.ecc_cost(eng.ctx, scan.id, Bn, th.data_ptr(), params, cost.data_ptr(), pairs.data_ptr(), ws.data_ptr(),
                       ws.numel(), stream)
        torch.cuda.synchronize(dev)
        out.append((cost.cpu().numpy(), pairs.cpu().numpy()))
    return out


def test_noalloc_equals_workspace_entry_two_calls(eng):
    g_big, big = _scan(eng, 48, 21)
    g_small, small = _scan(eng, 16, 22)
    cases = [
        ("48 views, B = 4, K = 100, c = 40, FP64 geometry", big, g_big,
         inputs.random_motion(31, 4, 48), big.params(100, g_big.default_object_radius(), 40.0, "f64")),
        ("16 views, B = 1, K = 64", small, g_small,
         inputs.random_motion(32, 1, 16), small.params(64, g_small.default_object_radius())),
        ("48 views again, B = 3, K = 64, detector range", big, g_big,
         inputs.random_motion(33, 3, 48), big.params(64, g_big.default_object_radius(), kappa="detector")),
    ]
    for name, scan, g, theta, params in cases:
        _say(f"case: noalloc vs workspace, {name}")
        (c_ws, p_ws), (c_na, p_na) = _both(eng, scan, theta, params)
        assert np.all(np.isfinite(c_ws)) and np.all(np.isfinite(p_ws))
        assert np.array_equal(c_na, c_ws), (c_na, c_ws)
        assert np.array_equal(p_na, p_ws)
        _say(f"  costs {c_na}")
    big.free()
    small.free()


def test_noalloc_refuses_oversize_evaluation(eng):
    import torch

    _say("case: noalloc oversize request")
    g, scan = _scan(eng, 48, 23)
    Bn = 512
    need = B.ecc_workspace_bytes(eng.ctx, scan.id, Bn, 0)
    assert need > B.ECC_NOALLOC_SCRATCH_BYTES
    th = torch.zeros((Bn, 48, 6), dtype=torch.float64, device=eng.device)
    cost = torch.empty(Bn, dtype=torch.float64, device=eng.device)
    with pytest.raises(B.EccError) as ei:
        B.ecc_cost_noalloc(eng.ctx, scan.id, Bn, th.data_ptr(), scan.params(64, g.default_object_radius()),
                           cost.data_ptr(), 0, torch.cuda.current_stream(eng.device).cuda_stream)
    assert ei.value.status == B.ECC_E_ARG
    assert "scratch" in str(ei.value)
    # the largest B that fits still runs, and equals the workspace entry
    fit = max(b for b in range(1, Bn) if B.ecc_workspace_bytes(eng.ctx, scan.id, b, 0) <= B.ECC_NOALLOC_SCRATCH_BYTES)
    _say(f"  largest B within the scratch: {fit}")
    theta = inputs.random_motion(34, fit, 48)
    (c_ws, p_ws), (c_na, p_na) = _both(eng, scan, theta, scan.params(64, g.default_object_radius()))
    assert np.array_equal(c_na, c_ws) and np.array_equal(p_na, p_ws)
    scan.free()
