"""Pins of the oracle to the mathematics (see ``pins.py``): the looked-up
S along epipolar lines against closed-form 3-D Radon derivatives (Eq. 1's
weight, the fold sign, the bilinear cell), the hit test behind N_kappa (Eq.
15) against a line clip, the tangency of the object-sphere arc (Eq. 3), and
the cosine weight of Eq. 1 on a wide-cone sphere."""
import oracle

import pins


def test_lookup_matches_closed_form_radon_derivative():
    r = {}
    pins.check_lookup_closed_form(oracle, r)
    print(r)


def test_hit_test_matches_line_clip_and_counts_n_kappa():
    r = {}
    pins.check_hit_test(oracle, r)
    print(r)


def test_kappa_max_is_tangent_to_object_sphere():
    r = {}
    pins.check_kappa_max(oracle, r)
    print(r)


def test_cosine_weight_on_wide_cone_sphere():
    r = {}
    pins.check_cosine_weight(oracle, r)
    print(r)
