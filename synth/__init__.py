"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module produces *inputs only*: closed flat-triangle surface meshes and seeded
complex Gaussian probe blocks.  It contains none of the method's arithmetic (no
quadrature, no Green's function, no contour or Chebyshev nodes), so that the oracle
and the HIP path can both consume it without sharing any of the computation they are
compared on.

The paper's own meshes (a unit cube with 864 triangles, a unit sphere with 384
triangles, an industrial pump casing) are not available; the stand-ins are seeded
synthetic meshes of the same kind (closed, flat triangles, Dirichlet single layer):
icospheres at subdivision level L (20*4**L triangles) and perturbed variants, class-I
geodesic spheres of any frequency f (20*f**2 triangles) scaled to seeded ellipsoids, and
box surfaces meshed by uniform face grids.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "box_surface",
    "icosahedron",
    "icosphere",
    "perturbed_icosphere",
    "ellipsoid",
    "geodesic_sphere",
    "ellipsoid_batch",
    "probe_block",
    "mesh_edges_ok",
    "nearfield_samples",
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


def geodesic_sphere(freq: int):
    """Class-I geodesic sphere of frequency f: every icosahedron face carries the uniform
    triangular grid of its barycentric points (i, j, f - i - j) / f, each grid triangle
    keeps the face's orientation, and the grid points are projected radially onto the unit
    sphere.  Points on a shared icosahedron edge or vertex are created once (keyed by
    their nonzero barycentric weights on the icosahedron's vertices), so the surface is
    closed.  Returns (xyz float64 [10 f^2 + 2, 3], tri int32 [20 f^2, 3])."""
    f = int(freq)
    if f < 1:
        raise ValueError("frequency must be >= 1")
    v, faces = icosahedron()
    index: dict[tuple, int] = {}
    pts = []

    def vid(a, b, c, i, j):
        w = {a: f - i - j}
        w[b] = w.get(b, 0) + i
        w[c] = w.get(c, 0) + j
        key = tuple(sorted((k, x) for k, x in w.items() if x))
        k = index.get(key)
        if k is None:
            p = ((f - i - j) * v[a] + i * v[b] + j * v[c]) / f
            pts.append(p / np.linalg.norm(p))
            k = len(pts) - 1
            index[key] = k
        return k

    tris = []
    for a, b, c in faces:
        for i in range(f):
            for j in range(f - i):
                tris.append((vid(a, b, c, i, j), vid(a, b, c, i + 1, j), vid(a, b, c, i, j + 1)))
                if i + j < f - 1:
                    tris.append((vid(a, b, c, i + 1, j), vid(a, b, c, i + 1, j + 1), vid(a, b, c, i, j + 1)))
    return np.asarray(pts, dtype=np.float64), np.asarray(tris, dtype=np.int32)


def harmonic_sphere(freq: int = 158, seed: int = 5, amplitude: float = 0.1, lmax: int = 6):
    """Class-I geodesic sphere of frequency f (20 f^2 triangles; f = 158 gives 499,280) with
    each vertex moved radially to r = 1 + amplitude sum_{l <= lmax, |m| <= l} c_lm Y_lm, the
    Y_lm real orthonormal spherical harmonics and c_lm ~ N(0, 1)/sqrt(#terms) drawn from
    PCG64(seed) in (l, m) order: a smooth star-shaped closed surface of uneven curvature."""
    from scipy.special import sph_harm_y

    xyz, tri = geodesic_sphere(freq)
    theta = np.arccos(np.clip(xyz[:, 2], -1.0, 1.0))
    phi = np.arctan2(xyz[:, 1], xyz[:, 0])
    rng = np.random.Generator(np.random.PCG64(seed))
    terms = (lmax + 1) ** 2
    r = np.ones(len(xyz))
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            c = rng.standard_normal() / np.sqrt(terms)
            Y = sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                y = np.sqrt(2.0) * Y.real
            elif m < 0:
                y = np.sqrt(2.0) * Y.imag
            else:
                y = Y.real
            r += amplitude * c * y
    return xyz * r[:, None], tri


def ellipsoid_batch(count: int = 64, seed: int = 4, freq=(10, 44), axes=(0.5, 1.5), centre=(3.0, 7.0)):
    """A seeded batch of uneven ellipsoid meshes, each with the real centre of its own
    contour.  From NumPy's PCG64(seed), per mesh in order: the geodesic frequency
    f ~ U{freq[0] .. freq[1]} (20 f^2 triangles), three semi-axes ~ U[axes], and the
    centre ~ U[centre].  Returns a list of (xyz, tri, semi_axes, centre) tuples; meshes of
    equal frequency share one geodesic sphere before scaling."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cache: dict[int, tuple] = {}
    out = []
    for _ in range(int(count)):
        f = int(rng.integers(freq[0], freq[1] + 1))
        ax = rng.uniform(axes[0], axes[1], size=3)
        c = float(rng.uniform(centre[0], centre[1]))
        if f not in cache:
            cache[f] = geodesic_sphere(f)
        xyz, tri = cache[f]
        out.append((xyz * ax[None, :], tri, ax, c))
    return out


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


def _point_triangle_distance_2d(x, p, q):
    """Distance from points x (k x 3) to the triangles (0,0,0), (1,0,0), (p,q,0) (arrays of k)."""
    A = np.zeros((len(p), 3))
    B = np.zeros((len(p), 3))
    B[:, 0] = 1.0
    C = np.stack([p, q, np.zeros_like(p)], axis=1)

    def seg(a, b):
        d = b - a
        t = np.clip(np.einsum("ij,ij->i", x - a, d) / np.einsum("ij,ij->i", d, d), 0.0, 1.0)
        return np.linalg.norm(x - (a + t[:, None] * d), axis=1)

    # inside test of the projection by barycentric coordinates
    xp = x.copy()
    xp[:, 2] = 0.0
    v0, v1, v2 = B - A, C - A, xp - A
    d00 = np.einsum("ij,ij->i", v0, v0)
    d01 = np.einsum("ij,ij->i", v0, v1)
    d11 = np.einsum("ij,ij->i", v1, v1)
    d20 = np.einsum("ij,ij->i", v2, v0)
    d21 = np.einsum("ij,ij->i", v2, v1)
    den = d00 * d11 - d01 * d01
    lb = (d11 * d20 - d01 * d21) / den
    lc = (d00 * d21 - d01 * d20) / den
    inside = (lb >= 0.0) & (lc >= 0.0) & (lb + lc <= 1.0)
    out = np.minimum(np.minimum(seg(A, B), seg(B, C)), seg(C, A))
    return np.where(inside, np.abs(x[:, 2]), out)


def nearfield_samples(count: int, seed: int, dmin: float = 0.15, rmax: float = 2.0, kh_re=(0.0, 1.0),
                      kh_im=(-0.3, 0.3), min_angle_deg: float = 20.0, coplanar_frac: float = 0.5,
                      coplanar_w: float = 0.1):
    """Seeded (triangle, target, wavenumber) triples for training and validating the learned
    near-field correction, in the unit frame of a source triangle: A = (0,0,0), B = (1,0,0)
    (its longest edge, length 1), C = (p, q, 0) with p in [0, 1/2] and every angle at least
    `min_angle_deg` (p, q uniform over that region); the target uniform in the ball of radius
    `rmax` about the centroid (the near-pair test |x_a - x_b| < eta h_b with eta = rmax), with a
    fraction `coplanar_frac` moved to heights |w| <= coplanar_w (the neighbours on a smooth
    surface lie close to the plane), and at least `dmin` from the triangle; the wavenumber times
    the edge length uniform in the rectangle kh_re x kh_im.  Rejection sampling from
    numpy.random.PCG64(seed).  Returns P (count x 3 x 3), x (count x 3), kh (count, complex)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    tmin = np.tan(np.deg2rad(min_angle_deg))
    Ps, xs, ks = [], [], []
    have = 0
    while have < count:
        k = 4 * (count - have) + 64
        p = rng.uniform(0.0, 0.5, k)
        q = rng.uniform(0.0, 0.87, k)
        ok = (q <= np.sqrt(np.maximum(2.0 * p - p * p, 0.0))) & (q >= (1.0 - p) * tmin) & (q >= p * tmin)
        d = rng.normal(size=(k, 3))
        d /= np.linalg.norm(d, axis=1)[:, None]
        r = rmax * rng.uniform(0.0, 1.0, k) ** (1.0 / 3.0)
        cen = np.stack([(1.0 + p) / 3.0, q / 3.0, np.zeros(k)], axis=1)
        x = cen + r[:, None] * d
        flat = rng.uniform(0.0, 1.0, k) < coplanar_frac
        wz = rng.uniform(-coplanar_w, coplanar_w, k)
        x[:, 2] = np.where(flat, wz, x[:, 2])
        kr = rng.uniform(kh_re[0], kh_re[1], k)
        ki = rng.uniform(kh_im[0], kh_im[1], k)
        ok &= np.linalg.norm(x - cen, axis=1) < rmax
        ok &= _point_triangle_distance_2d(x, p, q) >= dmin
        idx = np.nonzero(ok)[0][: count - have]
        P = np.zeros((idx.size, 3, 3))
        P[:, 1, 0] = 1.0
        P[:, 2, 0] = p[idx]
        P[:, 2, 1] = q[idx]
        Ps.append(P)
        xs.append(x[idx])
        ks.append(kr[idx] + 1j * ki[idx])
        have += idx.size
    return np.concatenate(Ps), np.concatenate(xs), np.concatenate(ks)

