import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP engine")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the host")


@pytest.fixture(scope="session")
def small16():
    """The 16-view 128x128 scan (10-ellipsoid phantom, seed 1), with images of
    the phantom as drawn and of a variant whose ellipsoids all stay inside the
    field of view."""
    from paper_1806_02637_amd import inputs
    import oracle

    w = inputs.WORKLOADS["small16"]
    g = w.geom
    P = g.projection_matrices()
    intr = g.intrinsics()
    grid = oracle.SinoGrid(g.W, g.H, w.n_alpha, w.n_t, w.ds_px)
    imgs = inputs.project(g, w.phantom())
    imgs_c = inputs.project(g, w.phantom(contained=True))
    sino = oracle.FullSinograms.build(imgs, grid, intr)
    sino_c = oracle.FullSinograms.build(imgs_c, grid, intr)
    params = oracle.EccParams(w.K, w.R_mm)
    return dict(w=w, geom=g, P=P, intr=intr, grid=grid, images=imgs, images_c=imgs_c, sino=sino,
                sino_c=sino_c, params=params)


@pytest.fixture(scope="session")
def rng():
    return np.random.default_rng(12345)
