"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module produces *inputs only*: closed flat-triangle surface meshes and seeded
complex Gaussian probe blocks.  It contains none of the method's arithmetic (no
quadrature, no Green's function, no contour or Chebyshev nodes), so that the oracle
and the HIP path can both consume it without sharing any of the computation they are
compared on.

The paper's own meshes (a unit cube with 864 triangles, a unit sphere with 384
triangles, an industrial pump casing) are not available; the stand-ins are seeded
synthetic meshes of the same kind (closed, flat triangles, Dirichlet single layer):
icospheres at subdivision level L (20*4**L triangles) and perturbed variants, and box
surfaces meshed by uniform face grids.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "box_surface",
    "icosahedron",
    "icosphere",
    "perturbed_icosphere",
    "ellipsoid",
    "probe_block",
    "mesh_edges_ok",
]


def icosahedron():
    """Regular icosahedron inscribed in the unit sphere (12 vertices, 20 faces, outward CCW)."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array(
        [
            [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
            [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
            [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1],
        ],
        dtype=np.float64,
    )
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array(
        [
            [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
            [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
            [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
            [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
        ],
        dtype=np.int32,
    )
    return v, f


def icosphere(level: int):
    """Unit icosphere: the icosahedron split `level` times into four, vertices projected
    radially onto the unit sphere.  Returns (xyz float64 [nv,3], tri int32 [n,3]) with
    nv = 10*4**level + 2 and n = 20*4**level."""
    if level < 0:
        raise ValueError("level must be >= 0")
    v, f = icosahedron()
    verts = [tuple(x) for x in v]
    faces = f.tolist()
    for _ in range(level):
        cache: dict[tuple[int, int], int] = {}

        def mid(i: int, j: int) -> int:
            key = (i, j) if i < j else (j, i)
            k = cache.get(key)
            if k is None:
                p = np.add(verts[i], verts[j]) * 0.5
                p = p / np.linalg.norm(p)
                verts.append(tuple(p))
                k = len(verts) - 1
                cache[key] = k
            return k

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        faces = nf
    return np.asarray(verts, dtype=np.float64), np.asarray(faces, dtype=np.int32)


def perturbed_icosphere(level: int, amplitude: float, seed: int):
    """Icosphere whose vertices are moved tangentially by a seeded random displacement of
    relative size `amplitude` (times the local edge length) and re-projected onto the
    unit sphere: a closed sphere mesh with uneven triangle areas."""
    xyz, tri = icosphere(level)
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 1.1 / (2 ** level)  # icosahedron edge ~1.05, halved per level
    d = rng.standard_normal(xyz.shape) * (amplitude * h)
    d -= (d * xyz).sum(axis=1, keepdims=True) * xyz  # tangential part
    p = xyz + d
    p /= np.linalg.norm(p, axis=1, keepdims=True)
    return p, tri


def ellipsoid(level: int, semi_axes):
    """Icosphere scaled to an ellipsoid with the given semi-axes (ax, ay, az)."""
    xyz, tri = icosphere(level)
    return xyz * np.asarray(semi_axes, dtype=np.float64)[None, :], tri


def box_surface(dims=(1.0, 0.8, 0.6), counts=(126, 101, 76)):
    """Surface of the box [0, a] x [0, b] x [0, c] (dims) on the uniform grid with
    counts = (nx, ny, nz) intervals per edge direction: every face square is split into two
    triangles along one diagonal, so n = 4 (nx ny + nx nz + ny nz) triangles sharing the
    grid vertices (watertight).  The default is the 1.0 x 0.8 x 0.6 box with 119,912
    triangles."""
    nx, ny, nz = (int(c) for c in counts)
    a, b, c = (float(d) for d in dims)
    index = -np.ones((nx + 1, ny + 1, nz + 1), dtype=np.int64)
    pts = []

    def vid(i, j, k):
        if index[i, j, k] < 0:
            index[i, j, k] = len(pts)
            pts.append((a * i / nx, b * j / ny, c * k / nz))
        return index[i, j, k]

    tris = []

    def face(fix_axis, fix_val, u_axis, nu, v_axis, nv):
        for iu in range(nu):
            for iv in range(nv):
                corners = []
                for du, dv in ((0, 0), (1, 0), (1, 1), (0, 1)):
                    ijk = [0, 0, 0]
                    ijk[fix_axis] = fix_val
                    ijk[u_axis] = iu + du
                    ijk[v_axis] = iv + dv
                    corners.append(vid(*ijk))
                tris.append((corners[0], corners[1], corners[2]))
                tris.append((corners[0], corners[2], corners[3]))

    for val, n_fix in ((0, None), (1, None)):
        face(2, 0 if val == 0 else nz, 0, nx, 1, ny)
        face(1, 0 if val == 0 else ny, 0, nx, 2, nz)
        face(0, 0 if val == 0 else nx, 1, ny, 2, nz)
    return np.asarray(pts, dtype=np.float64), np.asarray(tris, dtype=np.int32)


def probe_block(n: int, m: int, seed: int) -> np.ndarray:
    """Seeded complex Gaussian probe block V = (X + iY)/sqrt(2), X, Y ~ N(0,1) i.i.d.,
    drawn from NumPy's PCG64(seed); shape (n, m), complex128, C-contiguous."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.standard_normal((n, m, 2))
    v = (x[..., 0] + 1j * x[..., 1]) / np.sqrt(2.0)
    return np.ascontiguousarray(v.astype(np.complex128))


def mesh_edges_ok(tri: np.ndarray) -> bool:
    """True when every undirected edge belongs to exactly two faces (closed surface)."""
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    e = np.sort(e, axis=1)
    _, counts = np.unique(e, axis=0, return_counts=True)
    return bool(np.all(counts == 2))
