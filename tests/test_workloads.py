"""Seeded geometry generators shared by the oracle and the device path."""
import numpy as np

from paper_2403_01566_amd import workloads as W


def test_cube_surface_closed_form_m1():
    P, N = W.cube_surface(1)
    assert P.shape == (12, 3) and N.shape == (12, 3)
    # face +z is the sixth face: its two triangles have in-plane centroids
    # (1/3, -1/3) and (-1/3, 1/3)
    assert np.allclose(P[10], [1 / 3, -1 / 3, 1.0]) and np.allclose(P[11], [-1 / 3, 1 / 3, 1.0])
    assert np.array_equal(N[10], [0.0, 0.0, 1.0])
    assert np.array_equal(N[0], [-1.0, 0.0, 0.0])


def test_cube_surface_invariants():
    for m in (2, 5, 16):
        P, N = W.cube_surface(m)
        assert P.shape == (12 * m * m, 3)
        assert np.allclose(np.abs(P).max(axis=1), 1.0)                   # on the surface
        assert np.allclose((P * N).sum(axis=1), 1.0)                      # outward unit normals
        assert np.allclose(np.linalg.norm(N, axis=1), 1.0)
        assert len(np.unique(P.round(12), axis=0)) == len(P)              # distinct
        assert np.allclose(P.mean(axis=0), 0.0)                           # symmetric
        # every face holds 2 m^2 centroids, inside the face
        for axis in range(3):
            for sign in (-1.0, 1.0):
                on = np.isclose(P[:, axis], sign) & (N[:, axis] == sign)
                assert on.sum() == 2 * m * m
                assert np.all(np.abs(np.delete(P[on], axis, axis=1)) < 1.0)


def test_start_vector_is_seeded():
    a, b, c = W.start_vector(100, 7), W.start_vector(100, 7), W.start_vector(100, 8)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
