"""Seeded synthetic point sets for the H2 product workloads.

This module only generates geometry (points, normals, per-instance parameters).
It holds none of the method's arithmetic, so both the HIP path and the FP64
oracle may take their inputs from it.

Workloads (stand-ins for the paper's Galerkin meshes, Section 6):
  * ``grid2d(m)``: m x m cell-centred grid in [0,1]^2, point (i+1/2, j+1/2)/m,
    index i + m*j (x index fastest).
  * ``uniform2d(n, seed)``: n uniform random points in [0,1]^2 (PCG64).
  * ``icosphere(level)``: icosahedron refined ``level`` times by edge
    midpoints projected to the unit sphere; returns the 20*4^level triangle
    centroids (not projected) and the outward unit face normals.
  * ``fibsphere(n)``: Fibonacci lattice on the unit sphere; normals = points.
  * ``batched_instances``, ``serving_requests``, ``serving_points``: the
    parameters of the many-products and the serving workloads (seeded).
  * ``cube_surface(m)``: surface of [-1,1]^3, every face cut into m x m
    squares and every square into two triangles; returns the 12*m^2 triangle
    centroids and the outward face normals (the double-layer geometry of the
    paper's experiments: n = 3072 for m = 16, 6912 for m = 24, ...).
"""
from __future__ import annotations

import math

import numpy as np


def grid2d(m: int = 32) -> np.ndarray:
    i = np.arange(m, dtype=np.float64)
    x = (i + 0.5) / m
    pts = np.empty((m * m, 2), dtype=np.float64)
    # index i + m*j: x fastest
    pts[:, 0] = np.tile(x, m)
    pts[:, 1] = np.repeat(x, m)
    return pts


def uniform2d(n: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.random((n, 2))


def _icosahedron():
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    v = []
    for a in (-1.0, 1.0):
        for b in (-phi, phi):
            v.append((0.0, a, b))
            v.append((a, b, 0.0))
            v.append((b, 0.0, a))
    v = np.array(v, dtype=np.float64)
    # faces: triples of mutually adjacent vertices (edge length 2)
    nv = len(v)
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=2)
    adj = np.abs(d - 2.0) < 1e-9
    faces = []
    for a in range(nv):
        for b in range(a + 1, nv):
            if not adj[a, b]:
                continue
            for c in range(b + 1, nv):
                if adj[a, c] and adj[b, c]:
                    faces.append((a, b, c))
    assert len(faces) == 20
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = []
    for a, b, c in faces:
        n = np.cross(v[b] - v[a], v[c] - v[a])
        if np.dot(n, v[a] + v[b] + v[c]) < 0:
            b, c = c, b
        f.append((a, b, c))
    return v, np.array(f, dtype=np.int64)


def icosphere(level: int):
    """Returns (centroids [n,3], normals [n,3]) with n = 20*4**level."""
    v, f = _icosahedron()
    verts = [tuple(x) for x in v]
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                p = np.array(verts[a]) + np.array(verts[b])
                p /= np.linalg.norm(p)
                idx = len(verts)
                verts.append(tuple(p))
                cache[key] = idx
            return idx

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf.append((a, ab, ca))
            nf.append((ab, b, bc))
            nf.append((ca, bc, c))
            nf.append((ab, bc, ca))
        f = np.array(nf, dtype=np.int64)
    V = np.array(verts, dtype=np.float64)
    A, B, C = V[f[:, 0]], V[f[:, 1]], V[f[:, 2]]
    cen = (A + B + C) / 3.0
    nrm = np.cross(B - A, C - A)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    # orient outward
    sgn = np.sign(np.einsum("ij,ij->i", nrm, cen))
    nrm *= sgn[:, None]
    return cen, nrm


def cube_surface(m: int):
    """Returns (centroids [12 m^2, 3], outward unit normals [12 m^2, 3]).
    Face order -x, +x, -y, +y, -z, +z; on a face the two in-plane axes run in
    increasing index order, squares row-major; each square (lower-left corner
    (u, v), side h = 2/m) gives the triangles (u,v),(u+h,v),(u+h,v+h) and
    (u,v),(u+h,v+h),(u,v+h), with centroids at (u + 2h/3, v + h/3) and
    (u + h/3, v + 2h/3)."""
    h = 2.0 / m
    g = -1.0 + h * np.arange(m, dtype=np.float64)
    U, V = np.meshgrid(g, g, indexing="ij")
    U, V = U.ravel(), V.ravel()
    tri = np.stack([np.stack([U + 2 * h / 3, V + h / 3], 1), np.stack([U + h / 3, V + 2 * h / 3], 1)], 1)
    tri = tri.reshape(-1, 2)  # 2 m^2 in-plane centroids, the two triangles of a square adjacent
    cen, nrm = [], []
    for axis in range(3):
        others = [a for a in range(3) if a != axis]
        for sign in (-1.0, 1.0):
            c = np.empty((tri.shape[0], 3))
            c[:, axis] = sign
            c[:, others[0]] = tri[:, 0]
            c[:, others[1]] = tri[:, 1]
            nv = np.zeros((tri.shape[0], 3))
            nv[:, axis] = sign
            cen.append(c)
            nrm.append(nv)
    return np.concatenate(cen), np.concatenate(nrm)


def fibsphere(n: int):
    i = np.arange(n, dtype=np.float64) + 0.5
    z = 1.0 - 2.0 * i / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    ga = math.pi * (3.0 - math.sqrt(5.0))
    th = ga * i
    pts = np.stack([r * np.cos(th), r * np.sin(th), z], axis=1)
    return pts, pts.copy()


def batched_instances(count: int = 64, seed: int = 2403):
    """Parameters of the many-products workload: n_i log-uniform in
    [1024, 32768], Chebyshev order p_i in {3,4,5,6}, uniform points."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(1024), math.log(32768)))))
        p = int(rng.integers(3, 7))
        pseed = int(rng.integers(0, 2**31 - 1))
        out.append({"n": n, "order": p, "leaf": 32 if p <= 4 else 64, "points_seed": pseed})
    return out


def serving_requests(count: int, rate: float = 200.0, seed: int = 2404, m_range=(12, 17)):
    """Seeded request stream of the serving workload: Poisson arrivals (mean
    `rate` per second; times in seconds from 0), each request picks the
    geometry ("2d": uniform points in [0,1]^2, or "sphere": Fibonacci lattice),
    n = 2^m with m uniform in m_range, the Chebyshev order (2D: 3..8, sphere:
    3..4) and eps in {1e-4, 1e-6, 1e-8}, all uniformly."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for _ in range(count):
        t += rng.exponential(1.0 / rate)
        geo = "2d" if rng.integers(0, 2) == 0 else "sphere"
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        p = int(rng.integers(3, 9)) if geo == "2d" else int(rng.integers(3, 5))
        eps = float([1e-4, 1e-6, 1e-8][int(rng.integers(0, 3))])
        out.append({"t": t, "geometry": geo, "m": m, "order": p, "eps": eps})
    return out


def serving_points(geometry: str, m: int):
    """Points (and normals or None) of a serving operand: 2D uniform points
    with seed 2405 + m, or the Fibonacci sphere with 2^m points."""
    if geometry == "2d":
        return uniform2d(2 ** m, 2405 + m), None
    return fibsphere(2 ** m)


def start_vector(n: int, seed: int) -> np.ndarray:
    """Seeded standard-normal start vector of the power iteration (n entries,
    original point order)."""
    return np.random.Generator(np.random.PCG64(seed)).standard_normal(n)
