"""The algebra behind the tangent-frame form of the dual step (CPU, FP64).

The fused kernels carry the dual variable p in each pixel's orthonormal frame
U = [e1 e2 n] of the surface (x, y, tau(x, y)) and use M = [e1 e2] T with an
upper-triangular T (Section 3.1, eqn. (3) for M).  These checks pin the
identities that make that form the same iteration: orthonormality, the
factorisation of M (with masked columns), M^T p = T^T (U^T p)[:2], the dual
ascent in frame coordinates, and the invariance of the projection onto the
ball of radius sqrt(G).  They restate the formulas in numpy; the kernels'
own results are compared with the oracle in the GPU tests.
"""
import numpy as np
import pytest


def metric(tx, ty):
    G = 1.0 + tx * tx + ty * ty
    return np.array([[1 + ty * ty, -tx * ty], [-tx * ty, 1 + tx * tx], [tx, ty]]) / G, G


def frame(tx, ty):
    a = np.sqrt(1.0 + ty * ty)
    s = np.sqrt(1.0 + tx * tx + ty * ty)
    e1 = np.array([1 + ty * ty, -tx * ty, tx]) / (a * s)
    e2 = np.array([0.0, 1.0, ty]) / a
    n = np.array([-tx, -ty, 1.0]) / s
    T = np.array([[e1[0], e1[1]], [0.0, e2[1]]])
    return np.stack([e1, e2, n], axis=1), T, s


CASES = [(0.0, 0.0), (0.3, -1.7), (-12.0, 5.0), (250.0, 0.01), (1e-4, 3e3), (-0.5, -0.5)]


@pytest.mark.parametrize("tx,ty", CASES)
def test_frame_is_orthonormal_and_factors_the_metric(tx, ty):
    U, T, s = frame(tx, ty)
    M, G = metric(tx, ty)
    assert np.allclose(U.T @ U, np.eye(3), atol=1e-12)
    assert np.isclose(s * s, G, rtol=1e-14)
    assert np.allclose(U[:, :2] @ T, M, rtol=1e-12, atol=1e-15)
    # the normal is orthogonal to both columns of M (M^T n = 0)
    assert np.allclose(M.T @ U[:, 2], 0.0, atol=1e-12)
    # M^T M = g^{-1}: singular values 1 and 1/sqrt(G)
    sv = np.linalg.svd(M, compute_uv=False)
    assert np.allclose(sorted(sv), sorted([1.0, 1.0 / s]), rtol=1e-10)


@pytest.mark.parametrize("tx,ty", CASES)
@pytest.mark.parametrize("hx,hy", [(1, 1), (0, 1), (1, 0), (0, 0)])
def test_dual_step_in_frame_coordinates(tx, ty, hx, hy):
    rng = np.random.default_rng(7)
    U, T, s = frame(tx, ty)
    M, _ = metric(tx, ty)
    D = np.diag([hx, hy]).astype(float)  # masked columns at the image border
    sigma = 0.27
    for _ in range(20):
        p = rng.normal(size=3) * s
        g = rng.normal(size=2)
        pf = U.T @ p
        # q = M^T p from the first two frame coordinates only
        assert np.allclose((M @ D).T @ p, (T @ D).T @ pf[:2], rtol=1e-10, atol=1e-12)
        # ascent: U^T (p + sigma M D g) = p' + (sigma T D g, 0)
        pbar = p + sigma * (M @ D) @ g
        pbar_f = pf + np.concatenate([sigma * (T @ D) @ g, [0.0]])
        assert np.allclose(U.T @ pbar, pbar_f, rtol=1e-10, atol=1e-12)
        # projection onto the ball of radius s commutes with the rotation
        proj = lambda v: v / max(1.0, np.linalg.norm(v) / s)
        assert np.allclose(U @ proj(pbar_f), proj(pbar), rtol=1e-10, atol=1e-12)


def test_rotation_round_trip():
    rng = np.random.default_rng(3)
    for tx, ty in CASES:
        U, _, _ = frame(tx, ty)
        p = rng.normal(size=3)
        assert np.allclose(U @ (U.T @ p), p, atol=1e-12)
