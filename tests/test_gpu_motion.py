"""Motion-estimation loop (Sec. "Optimization") on the GPU: the Akima spline
kernels against the oracle's spline, and the L-BFGS loop recovering a smooth
out-of-plane drift from projections taken while the object moved."""
import math

import numpy as np
import pytest

from oracle import spline
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


def test_spline_kernels_match_oracle(eng):
    import torch

    from paper_1806_02637_amd.motion import SplineMotion

    _say("case: spline kernels vs oracle (N=60, 9 nodes and N=496, 17 nodes)")
    rng = np.random.default_rng(11)
    for n_views, n_nodes, Bn in ((60, 9, 3), (496, 17, 2)):
        g = inputs.ScanGeometry(n_views, 64, 48, 3.0)
        scan = eng.load_scan(g.projection_matrices(), g.intrinsics(), np.zeros((n_views, 48, 64), np.float32))
        model = SplineMotion(scan, n_nodes)
        nodes = rng.normal(0, 1.5, (Bn, 6, n_nodes))
        nodes[0, 2, 3:6] = 0.7  # a plateau (Akima's zero-weight branch)
        nodes_dev = torch.tensor(nodes, device="cuda")
        th = model.theta(nodes_dev).cpu().numpy()
        gth = rng.normal(size=(Bn, n_views, 6)).astype(np.float32)
        gn = model.grad(nodes_dev, torch.tensor(gth, device="cuda")).cpu().numpy()
        for b in range(Bn):
            ref = spline.spline_motion(model.node_x, nodes[b], n_views)
            assert np.abs(th[b] - ref).max() <= 1e-12 * (1 + np.abs(ref).max())
            gref = spline.spline_motion_grad(model.node_x, nodes[b], gth[b].astype(np.float64))
            assert np.abs(gn[b] - gref).max() <= 1e-11 * (1 + np.abs(gref).max())
        scan.free()


def test_spline_argument_errors(eng):
    import torch

    _say("case: spline argument errors")
    g = inputs.ScanGeometry(20, 32, 32, 3.0)
    nodes = torch.zeros((1, 6, 5), dtype=torch.float64, device="cuda")
    th = torch.empty((1, 20, 6), dtype=torch.float64, device="cuda")
    ctx = eng.ctx
    for nx in (np.array([0.0, 5.0, 5.0, 10.0, 19.0]), np.array([1.0, 5.0, 8.0, 10.0, 19.0]),
               np.array([0.0, 5.0, 8.0, 10.0, 18.0])):
        with pytest.raises(B.EccError) as ei:
            B.ecc_spline_motion(ctx, 1, 20, 5, np.ascontiguousarray(nx).ctypes.data, nodes.data_ptr(),
                                th.data_ptr(), 0)
        assert ei.value.status == B.ECC_E_ARG
    nx = np.linspace(0, 19, 2)
    with pytest.raises(B.EccError):
        B.ecc_spline_motion(ctx, 1, 20, 2, nx.ctypes.data, nodes.data_ptr(), th.data_ptr(), 0)
    del g


@pytest.mark.parametrize("kappa", ["object", "detector"])
def test_motion_estimation_recovers_drift(eng, kappa):
    """A 96-view scan (620x480 detector at 0.616 mm) of an FOV-contained
    phantom drifting along z (2 mm peak): L-BFGS over 9 Akima nodes of t_z
    lowers the cost by orders of magnitude and recovers the drift (up to the
    common offset, which the cost cannot see) to a fraction of a pixel, with
    either reading of the sampled plane range."""
    import torch

    from paper_1806_02637_amd.motion import estimate_motion

    _say(f"case: motion estimation 96 views, 9 t_z nodes, {kappa} range")
    g = inputs.ScanGeometry(96, 620, 480, 0.616)
    truth = inputs.smooth_motion(21, g.n_views, peak=2.0, params=(5,))
    phantom = inputs.random_phantom(2, 30, contained_radius=0.95 * g.fov_radius())
    imgs = inputs.project(g, phantom, device="cuda", as_tensor=True, motion=truth)
    scan = eng.load_scan(g.projection_matrices(), g.intrinsics(), imgs)
    scan.build_sinograms(360, 512, 0.5, "f32")
    del imgs
    torch.cuda.empty_cache()
    R = g.default_object_radius()
    c_true = float(scan.cost(truth[None], 256, R, kappa=kappa)[0])
    res = estimate_motion(scan, K=256, R_mm=R, n_nodes=9, params=(5,), max_iter=80, kappa=kappa)
    err0 = truth[:, 5] - truth[:, 5].mean()
    est = res.theta[:, 5] - res.theta[:, 5].mean()
    rms0, rms = float(np.sqrt(np.mean(err0 ** 2))), float(np.sqrt(np.mean((est - err0) ** 2)))
    _say(f"  cost {res.cost0:.4g} -> {res.cost:.4g} (truth {c_true:.4g}); {res.n_iter} iterations, "
         f"{res.n_evals} evaluations, {np.median(res.eval_ms):.2f} ms each; t_z RMS error {rms0:.3f} -> {rms:.3f} mm")
    # the 9-node spline cannot follow the drift exactly (it is not a spline),
    # so the cost ends near, not below, the cost at the true motion
    assert res.cost < 0.01 * res.cost0
    assert res.cost < 4.0 * c_true
    assert rms < 0.1 * rms0
    # the estimate is a real motion: other parameters untouched
    assert np.all(res.theta[:, :5] == 0.0)
    scan.free()
    assert math.isfinite(res.seconds)
