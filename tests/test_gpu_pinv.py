"""The pseudo-inverse route (the method the paper replaces) against the
method on the GPU: the same lines up to a positive scale, so the same cost to
rounding (the paper reports equal results for the two routes, Sec.
"Experiments")."""
import numpy as np
import pytest

import oracle
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


def test_pinv_route_matches_method_and_oracle_small16(eng, small16):
    from paper_1806_02637_amd.pinv import PinvRoute

    _say("case: pinv route small16 (oracle sinograms), B=3")
    s = small16
    g = s["geom"]
    scan = eng.load_scan(s["P"], s["intr"], s["images"])
    scan.set_sinograms(s["sino"].data)
    thetas = inputs.random_motion(1001, 3, g.n_views)
    route = PinvRoute(scan, s["P"], 3)
    c_pinv = route.cost(thetas, s["params"].K, s["params"].R_mm).cpu().numpy()
    c_meth = scan.cost(thetas, s["params"].K, s["params"].R_mm).cpu().numpy()
    for h in range(3):
        c_ref = oracle.ecc_cost(s["P"], s["intr"], thetas[h], s["grid"], s["sino"], s["params"])[0]
        _say(f"  hyp {h}: pinv vs method {abs(c_pinv[h] - c_meth[h]) / c_meth[h]:.2e}, "
             f"pinv vs oracle {abs(c_pinv[h] - c_ref) / c_ref:.2e}")
        assert abs(c_pinv[h] - c_meth[h]) <= 2e-6 * c_meth[h]
        assert abs(c_pinv[h] - c_ref) <= 1e-5 * c_ref
    scan.free()


def test_pinv_route_matches_method_per_pair(eng):
    from paper_1806_02637_amd.pinv import PinvRoute

    _say("case: pinv route 96 views 620x480, B=4, per pair")
    g = inputs.ScanGeometry(96, 620, 480, 0.616)
    P = g.projection_matrices()
    imgs = inputs.project(g, inputs.random_phantom(2, 30), device="cuda", as_tensor=True)
    scan = eng.load_scan(P, g.intrinsics(), imgs)
    scan.build_sinograms(360, 512, 0.5, "f32")
    del imgs
    thetas = inputs.random_motion(1002, 4, g.n_views)
    R = g.default_object_radius()
    route = PinvRoute(scan, P, 4)
    c_pinv, e_pinv = route.cost(thetas, 256, R, with_pairs=True)
    c_meth, e_meth = scan.cost(thetas, 256, R, with_pairs=True)
    c_pinv, c_meth = c_pinv.cpu().numpy(), c_meth.cpu().numpy()
    e_pinv, e_meth = e_pinv.cpu().numpy(), e_meth.cpu().numpy()
    rel = np.abs(e_pinv - e_meth) / np.maximum(e_meth, 1e-30)
    _say(f"  totals max rel {np.max(np.abs(c_pinv - c_meth) / c_meth):.2e}; "
         f"pairs median {np.median(rel):.2e} max {rel.max():.2e}")
    # both routes give the FP64 line maps up to a positive scale; rounded to
    # FP32 after normalisation they differ in the last bit, which moves a
    # pair's e by ~1e-6 typically and by up to ~1e-4 on nearly consistent
    # pairs (small e against large S values)
    assert np.all(np.abs(c_pinv - c_meth) <= 2e-6 * c_meth)
    assert np.median(rel) <= 1e-5 and np.quantile(rel, 0.999) <= 2e-4 and rel.max() <= 1e-3
    with pytest.raises(B.EccError) as ei:
        ws = scan.workspace(1, False)
        B.ecc_cost_pinv(scan.ctx, scan.id, 1, route.dev.data_ptr(), 0, scan.params(256, R),
                        route.dev.data_ptr(), 0, ws.data_ptr(), ws.numel(), 0)
    assert ei.value.status == B.ECC_E_ARG
    scan.free()
