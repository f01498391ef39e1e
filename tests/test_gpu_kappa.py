"""The detector-bounded plane range (ECC_KAPPA_DETECTOR) on the GPU against
the FP64 oracle: each pair samples the arc of the pencil around kappa = 0
whose lines meet both detectors (cost and gradient).  Hypotheses cover the
three kinds of pair arc: partial, the whole half circle (a source
projecting onto the other view's detector) including a partial arc reaching
past +-pi/2, and empty (a view moved 900 mm along the rotation axis: e = 0).  Bars as the
object-sphere range: 1e-5 relative on totals, 2e-4 relative plus 1e-5 of
the largest e per pair; an empty pair is exactly 0."""
import math

import numpy as np
import pytest

import oracle
from oracle.ecc import as_rows, pair_kappa_arc, pair_list
from oracle.geometry import moved_projection, pencil, source_position
from paper_1806_02637_amd import binding as B
from paper_1806_02637_amd import inputs

pytestmark = pytest.mark.gpu

FULL = (-0.5 * math.pi, 0.5 * math.pi)


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


def _hypotheses(n_views):
    rng = np.random.default_rng(0)
    wild = np.concatenate([rng.normal(0, 5, (n_views, 3)), rng.normal(0, 60, (n_views, 3))], 1)[None]
    far = 6.0 * inputs.random_motion(1002, 1, n_views)
    far[0, 5, 5] += 900.0
    return np.concatenate([np.zeros((1, n_views, 6)), inputs.random_motion(1001, 2, n_views), wild, far])


def _arc_kinds(P, intr, theta, W, H, R):
    kinds = dict(none=0, part=0, full=0, wide=0)
    for a, b in pair_list(len(P)):
        Pa, Pb = moved_projection(as_rows(P[a]), list(theta[a])), moved_projection(as_rows(P[b]), list(theta[b]))
        C_a, C_b = source_position(Pa), source_position(Pb)
        u1, u2, _ = pencil(C_a, C_b, R)
        arc = pair_kappa_arc(Pa, Pb, C_a, u1, u2, (intr[a], intr[b], W, H))
        if arc is None:
            kinds["none"] += 1
        elif arc == FULL:
            kinds["full"] += 1
        else:
            kinds["part"] += 1
            kinds["wide"] += arc[0] < -0.5 * math.pi or arc[1] > 0.5 * math.pi
    return kinds


@pytest.mark.parametrize("geom", ["f32", "f64"])
def test_detector_range_small16(eng, small16, geom):
    _say(f"case: detector kappa range small16 oracle sinograms geom={geom}")
    s = small16
    w, g = s["w"], s["geom"]
    scan = eng.load_scan(s["P"], s["intr"], s["images"])
    scan.set_sinograms(s["sino"].data.astype(np.float32), "f32")
    sino32 = oracle.FullSinograms(s["sino"].data.astype(np.float32).astype(np.float64), s["grid"])
    thetas = _hypotheses(g.n_views)
    params = oracle.EccParams(w.K, w.R_mm, kappa_range="detector")
    cost, pairs = scan.cost(thetas, w.K, w.R_mm, geom=geom, with_pairs=True, kappa="detector")
    cost, pairs = cost.cpu().numpy(), pairs.cpu().numpy()
    seen = dict(none=0, part=0, full=0, wide=0)
    for h in range(thetas.shape[0]):
        c_ref, e_ref, _, N = oracle.ecc_cost(s["P"], s["intr"], thetas[h], s["grid"], sino32, params)
        _say(f"  hyp {h}: {cost[h]:.9e} vs {c_ref:.9e}")
        assert abs(cost[h] - c_ref) <= 1e-5 * abs(c_ref), (h, cost[h], c_ref)
        tol = 2e-4 * np.abs(e_ref) + 1e-5 * np.abs(e_ref).max()
        assert np.all(np.abs(pairs[h] - e_ref) <= tol), (h, np.abs(pairs[h] - e_ref).max())
        assert np.all(pairs[h][N == 0] == 0.0)
        for k, v in _arc_kinds(s["P"], s["intr"], thetas[h], g.W, g.H, w.R_mm).items():
            seen[k] += v
    assert min(seen.values()) > 0, seen
    # the range differs from the object sphere's: the two costs differ
    obj = scan.cost(thetas[:1], w.K, w.R_mm, geom=geom).cpu().numpy()[0]
    assert abs(obj - cost[0]) > 1e-3 * abs(cost[0])
    scan.free()


def test_detector_range_pinv_route(eng, small16):
    """The pseudo-inverse route's lines are the same lines up to a positive
    scale, so their arcs and costs agree with the method's to rounding."""
    from paper_1806_02637_amd.pinv import PinvRoute

    _say("case: detector kappa range through the pseudo-inverse route")
    s = small16
    w, g = s["w"], s["geom"]
    scan = eng.load_scan(s["P"], s["intr"], s["images"])
    scan.set_sinograms(s["sino"].data.astype(np.float32), "f32")
    thetas = _hypotheses(g.n_views)
    route = PinvRoute(scan, s["P"], thetas.shape[0])
    a = scan.cost(thetas, w.K, w.R_mm, kappa="detector").cpu().numpy()
    b = route.cost(thetas, w.K, w.R_mm, kappa="detector").cpu().numpy()
    assert np.allclose(a, b, rtol=1e-5, atol=0.0), (a, b)
    scan.free()


def test_detector_range_gradient(eng, small16):
    """Adjoint with the detector-bounded range against the oracle's exact
    gradient (which follows each arc end as the zero angle of the corner
    that fixes it); the same bars as the object-sphere adjoint."""
    _say("case: detector kappa range gradient small16 vs oracle")
    s = small16
    w, g = s["w"], s["geom"]
    scan = eng.load_scan(s["P"], s["intr"], s["images"])
    scan.set_sinograms(s["sino"].data.astype(np.float32), "f32")
    sino32 = oracle.FullSinograms(s["sino"].data.astype(np.float32).astype(np.float64), s["grid"])
    thetas = _hypotheses(g.n_views)
    for c in (math.inf, 30.0):
        params = oracle.EccParams(w.K, w.R_mm, c, kappa_range="detector")
        cost, grad, pg = scan.cost_grad(thetas, w.K, w.R_mm, c=c, with_pair_grads=True, kappa="detector")
        cost_f = scan.cost(thetas, w.K, w.R_mm, c=c, kappa="detector")
        assert np.allclose(cost.cpu().numpy(), cost_f.cpu().numpy(), rtol=1e-6, atol=0)
        grad, pg = grad.cpu().numpy(), pg.cpu().numpy()
        for h in range(thetas.shape[0]):
            c_ref, g_ref, pg_ref = oracle.ecc_grad(s["P"], s["intr"], thetas[h], s["grid"], sino32, params)
            err = np.linalg.norm(grad[h] - g_ref) / np.linalg.norm(g_ref)
            _say(f"  c={c} hyp {h}: grad rel L2 {err:.2e}")
            assert err <= 2e-4
            nrm = np.linalg.norm(pg_ref, axis=1) + 1e-30
            perr = np.linalg.norm(pg[h] - pg_ref, axis=1) / nrm
            live = np.linalg.norm(pg_ref, axis=1) > 0
            assert np.all(pg[h][~live] == 0.0)
            assert np.quantile(perr[live], 0.99) <= 1e-3 and perr[live].max() <= 1e-2, perr[live].max()
    scan.free()


def test_detector_range_argument_errors(eng, small16):
    import torch

    _say("case: detector kappa range argument errors")
    s = small16
    g = s["geom"]
    scan = eng.load_scan(s["P"], s["intr"], s["images"])
    scan.set_sinograms(s["sino"].data.astype(np.float32), "f32")
    th = torch.zeros((1, g.n_views, 6), dtype=torch.float64, device="cuda")
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    ws = scan.workspace(1, True)
    for bad in (B.EvalParams(32, 0, 50.0, 0.0, 2, 0), B.EvalParams(32, 0, 50.0, 0.0, 0, 1)):
        with pytest.raises(B.EccError) as ei:
            B.ecc_cost(scan.ctx, scan.id, 1, th.data_ptr(), bad, out.data_ptr(), 0, ws.data_ptr(), ws.numel(), 0)
        assert ei.value.status == B.ECC_E_ARG
    with pytest.raises(ValueError):
        scan.params(32, 50.0, kappa="sphere")
    scan.free()
