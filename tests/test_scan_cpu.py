"""Host logic of the potential scan."""

import numpy as np

from paper_1202_2355_amd.scan import best_of


def test_best_of_is_the_vertex_of_the_parabola_through_the_minimum():
    v = np.array([0.8, 1.0, 1.2, 1.4, 1.6])
    c = 7.0 * (v - 1.13) ** 2 + 3.0
    assert abs(best_of(v, c) - 1.13) < 1e-12
    # uneven spacing
    v2 = np.array([0.5, 0.9, 1.0, 1.7])
    c2 = 2.0 * (v2 - 1.05) ** 2
    assert abs(best_of(v2, c2) - 1.05) < 1e-12


def test_best_of_at_the_ends_and_on_flat_data():
    v = np.array([1.0, 2.0, 3.0])
    assert best_of(v, [1.0, 2.0, 3.0]) == 1.0
    assert best_of(v, [3.0, 2.0, 1.0]) == 3.0
    # first minimum at 2; the parabola through (1, 2), (2, 1), (3, 1) has its vertex at 2.5
    assert abs(best_of(v, [2.0, 1.0, 1.0]) - 2.5) < 1e-12
