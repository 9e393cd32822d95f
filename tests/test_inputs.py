"""Seeded input generators: the links are SU(3), the smooth field has the
plaquette the workloads are quoted at, and the process-parallel generator
gives bitwise the same field as the serial one."""
import numpy as np

from paper_1701_07559_amd import inputs as I


def test_random_links_are_special_unitary():
    U = I.random_links((4, 2, 2, 6), 0.3, 11)
    m = U.reshape(-1, 3, 3)
    eye = np.eye(3)
    assert np.abs(m @ m.conj().transpose(0, 2, 1) - eye).max() < 1e-13
    assert np.abs(np.linalg.det(m) - 1.0).max() < 1e-13


def test_parallel_link_generation_is_bitwise_serial():
    dims = (6, 4, 4, 10)
    a = I.random_links(dims, 0.25, 202)
    b = I.random_links(dims, 0.25, 202, workers=3)
    assert np.array_equal(a, b)


def test_smooth_field_plaquette():
    # exp(i 0.25 H), E tr H^2 = 10: average plaquette in the range 0.6-0.7
    p = I.plaquette(I.random_links((6, 6, 6, 6), 0.25, 5))
    assert 0.6 < p < 0.7
