"""Parity of the HIP path with the FP64 oracle, through the C ABI.

Tolerances (FP32 path):
* sinogram cells: |GPU - oracle| <= 2e-5 * max |oracle| of the view (FP32
  positions and chunked FP32/FP64 sums of ~10^3 bilinear samples, then a
  central difference that cancels ~1 digit);
* total cost per hypothesis: 1e-5 relative;
* per-pair e: 2e-4 relative to the pair's own e plus 1e-5 of the largest e
  (e is a mean of squared differences of nearly equal values, so its relative
  error is the sinogram error amplified by |S| / |S_a - S_b|).
"""
import math

import numpy as np
import pytest

import oracle
from oracle.ecc import as_rows, ecc_pair, pair_index, pair_list
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


@pytest.fixture(scope="module")
def small(small16):
    return small16


def test_sinogram_parity_small16(eng, small):
    _say("case: sinogram small16 f32")
    w, g = small["w"], small["geom"]
    scan = eng.load_scan(small["P"], small["intr"], small["images"])
    scan.build_sinograms(w.n_alpha, w.n_t, w.ds_px, "f32")
    for v in range(g.n_views):
        got = scan.read_sinogram(v)
        ref = small["sino"].data[v]
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert err <= 2e-5, (v, err)
    scan.free()


@pytest.mark.parametrize("geom", ["f32", "f64"])
def test_cost_parity_small16_oracle_sinograms(eng, small, geom):
    # the oracle's own sinograms (cast to FP32) isolate geometry + lookup
    _say(f"case: cost small16 oracle sinograms geom={geom}")
    w, g = small["w"], small["geom"]
    scan = eng.load_scan(small["P"], small["intr"], small["images"])
    scan.set_sinograms(small["sino"].data.astype(np.float32), "f32")
    sino32 = oracle.FullSinograms(small["sino"].data.astype(np.float32).astype(np.float64), small["grid"])
    thetas = np.concatenate([np.zeros((1, g.n_views, 6)), inputs.random_motion(1001, 3, g.n_views)])
    cost, pairs = scan.cost(thetas, w.K, w.R_mm, geom=geom, with_pairs=True)
    cost, pairs = cost.cpu().numpy(), pairs.cpu().numpy()
    for h in range(thetas.shape[0]):
        c_ref, e_ref, _, _ = oracle.ecc_cost(small["P"], small["intr"], thetas[h], small["grid"], sino32,
                                             small["params"])
        assert abs(cost[h] - c_ref) <= 1e-5 * abs(c_ref), (h, cost[h], c_ref)
        tol = 2e-4 * np.abs(e_ref) + 1e-5 * np.abs(e_ref).max()
        assert np.all(np.abs(pairs[h] - e_ref) <= tol), (h, np.abs(pairs[h] - e_ref).max())
    scan.free()


def test_cost_parity_small16_end_to_end(eng, small):
    _say("case: cost small16 end to end")
    w, g = small["w"], small["geom"]
    scan = eng.load_scan(small["P"], small["intr"], small["images"])
    scan.build_sinograms(w.n_alpha, w.n_t, w.ds_px, "f32")
    thetas = np.concatenate([np.zeros((1, g.n_views, 6)), inputs.random_motion(1001, 2, g.n_views)])
    cost = scan.cost(thetas, w.K, w.R_mm).cpu().numpy()
    for h in range(thetas.shape[0]):
        c_ref = oracle.ecc_cost(small["P"], small["intr"], thetas[h], small["grid"], small["sino"],
                                small["params"])[0]
        assert abs(cost[h] - c_ref) <= 1e-5 * abs(c_ref), (h, cost[h], c_ref)
    scan.free()


def test_ragged_shapes_and_cauchy(eng):
    # 13 views = 78 pairs (one full 64-pair tile + 14), B = 5 (a partial group
    # of four hypotheses), K not a multiple of the wave width, finite c
    _say("case: ragged 13 views, B=5, K in (1, 100)")
    geom = inputs.ScanGeometry(13, 96, 80, 3.0)
    P, intr = geom.projection_matrices(), geom.intrinsics()
    imgs = inputs.project(geom, inputs.random_phantom(9, 6))
    grid = oracle.SinoGrid(geom.W, geom.H, 90, 97, 0.5)
    sino = oracle.FullSinograms.build(imgs, grid, intr)
    scan = eng.load_scan(P, intr, imgs)
    scan.set_sinograms(sino.data.astype(np.float32), "f32")
    sino32 = oracle.FullSinograms(sino.data.astype(np.float32).astype(np.float64), grid)
    thetas = inputs.random_motion(5, 5, geom.n_views)
    R = geom.default_object_radius()
    for K, c in ((100, math.inf), (1, math.inf), (64, 25.0)):
        cost, pairs = scan.cost(thetas, K, R, c=c, with_pairs=True)
        cost, pairs = cost.cpu().numpy(), pairs.cpu().numpy()
        for h in (0, 4):
            c_ref, e_ref, _, _ = oracle.ecc_cost(P, intr, thetas[h], grid, sino32, oracle.EccParams(K, R, c))
            assert abs(cost[h] - c_ref) <= 1e-5 * abs(c_ref) + 1e-12, (K, h, cost[h], c_ref)
            tol = 2e-4 * np.abs(e_ref) + 1e-5 * np.abs(e_ref).max()
            assert np.all(np.abs(pairs[h] - e_ref) <= tol), (K, h)
    scan.free()


def test_repeated_calls_are_bitwise_identical(eng, small):
    _say("case: determinism small16")
    w, g = small["w"], small["geom"]
    scan = eng.load_scan(small["P"], small["intr"], small["images"])
    scan.build_sinograms(w.n_alpha, w.n_t, w.ds_px, "f32")
    th = inputs.random_motion(77, 7, g.n_views)
    a, pa = scan.cost(th, w.K, w.R_mm, with_pairs=True)
    b, pb = scan.cost(th, w.K, w.R_mm, with_pairs=True)
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    assert np.array_equal(pa.cpu().numpy(), pb.cpu().numpy())
    # a hypothesis' result does not depend on its batch neighbours
    c1 = scan.cost(th[3:4], w.K, w.R_mm).cpu().numpy()
    assert c1[0] == a.cpu().numpy()[3]
    scan.free()


def _sampled_workload_check(eng, name, B, n_cells, n_pairs_check, seed, kappa="object"):
    """Full-size workload in the configuration the benchmark times: all B
    hypotheses evaluated on the GPU; sampled sinogram cells and sampled
    (hypothesis, pair) values recomputed one by one by the oracle from the
    same images."""
    import torch

    w = inputs.WORKLOADS[name]
    g = w.geom
    P, intr = g.projection_matrices(), g.intrinsics()
    imgs = inputs.project(g, w.phantom(), device="cuda", as_tensor=True)
    scan = eng.load_scan(P, intr, imgs)
    scan.build_sinograms(w.n_alpha, w.n_t, w.ds_px, "f32")
    thetas = w.motion(B)
    cost, pairs = scan.cost(thetas, w.K, w.R_mm, with_pairs=True, kappa=kappa)
    cost, pairs = cost.cpu().numpy(), pairs.cpu().numpy()
    rng = np.random.default_rng(seed)
    pair_ids = np.sort(rng.choice(w.n_pairs, n_pairs_check, replace=False))
    all_pairs = pair_list(g.n_views) if g.n_views <= 300 else None
    sel = []
    for pid in pair_ids:
        if all_pairs is not None:
            sel.append(all_pairs[pid])
        else:  # invert the triangle index
            a = 0
            while pair_index(a + 1, a + 2, g.n_views) <= pid:
                a += 1
            sel.append((a, int(pid - pair_index(a, a + 1, g.n_views)) + a + 1))
    views = sorted({v for ab in sel for v in ab} | set(rng.choice(g.n_views, 2, replace=False).tolist()))
    host = {v: imgs[v].cpu().numpy() for v in views}
    del imgs
    torch.cuda.empty_cache()

    class ViewImages:
        def __getitem__(self, v):
            return host[v]

    grid = oracle.SinoGrid(g.W, g.H, w.n_alpha, w.n_t, w.ds_px)
    lazy = oracle.LazySinograms(ViewImages(), grid, intr)
    # sampled sinogram cells
    for v in views[:3]:
        m = rng.integers(0, w.n_alpha + 1, n_cells)
        k = rng.integers(0, w.n_t, n_cells)
        got = scan.read_sinogram(v)[m, k]
        ref = lazy.cells(v, m, k)
        scale = np.abs(scan.read_sinogram(v)).max()
        assert np.abs(got - ref).max() <= 2e-5 * scale, (v, np.abs(got - ref).max() / scale)
    # sampled pairs, every hypothesis for the first pairs, two for the rest
    params = oracle.EccParams(w.K, w.R_mm, kappa_range=kappa)
    worst = 0.0
    for i, ((a, b), pid) in enumerate(zip(sel, pair_ids)):
        hyps = range(B) if i < 2 else (0, B - 1)
        for h in hyps:
            e_ref, _, _ = ecc_pair(as_rows(P[a]), as_rows(P[b]), list(thetas[h][a]), list(thetas[h][b]), intr[a],
                                   intr[b], grid, lazy, a, b, params)
            e_ref = float(e_ref)
            err = abs(pairs[h, pid] - e_ref)
            worst = max(worst, err / max(abs(e_ref), 1e-30))
            assert err <= 2e-4 * abs(e_ref) + 1e-7, (name, h, a, b, pairs[h, pid], e_ref)
    _say(f"{name} ({kappa} range): worst sampled pair rel err {worst:.2e}")
    # the total is the fixed-order sum of the per-pair values
    assert np.allclose(cost, pairs.astype(np.float64).sum(1), rtol=1e-6)
    scan.free()


def test_mid248_sampled_parity(eng):
    _say("case: mid248 sampled parity, B=32, K=256")
    _sampled_workload_check(eng, "mid248", 32, 400, 24, 11)


def test_full496_sampled_parity(eng):
    _say("case: full496 sampled parity, B=32, K=512")
    _sampled_workload_check(eng, "full496", 32, 200, 8, 12)


def test_full496_detector_range_sampled_parity(eng):
    _say("case: full496 sampled parity, detector-bounded plane range, B=32, K=512")
    _sampled_workload_check(eng, "full496", 32, 50, 4, 13, kappa="detector")
