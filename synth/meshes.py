"""Triangle meshes used as synthetic workloads.

Every generator returns ``(nodes, tris)`` with ``nodes`` a float64 array of
shape (V, 3) and ``tris`` an int32 array of shape (N, 3).  Triangles are
ordered counter-clockwise when seen from outside, so the right-hand normal
points away from the body (the mesh convention of the paper's appendix on
meshes).  The generators are deterministic; none of them uses randomness.
"""

import numpy as np


def _icosahedron():
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1],
    ], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    return v, f


def _orient_outward(nodes, tris):
    """Flip any triangle whose right-hand normal points towards the origin
    (valid for star-shaped bodies around the origin)."""
    p0, p1, p2 = nodes[tris[:, 0]], nodes[tris[:, 1]], nodes[tris[:, 2]]
    nrm = np.cross(p1 - p0, p2 - p0)
    c = p0 + p1 + p2
    bad = np.einsum("ij,ij->i", nrm, c) < 0
    tris = tris.copy()
    tris[bad] = tris[bad][:, [0, 2, 1]]
    return tris


def icosphere(subdiv, radius=1.0):
    """Recursively subdivided icosahedron: 20 * 4**subdiv triangles.

    Each step splits every triangle into four through its edge midpoints and
    projects the new vertices onto the sphere."""
    v, f = _icosahedron()
    verts = [tuple(p) for p in v]
    faces = f.tolist()
    for _ in range(subdiv):
        cache = {}
        new_faces = []

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                p = np.add(verts[a], verts[b]) * 0.5
                p = p / np.linalg.norm(p)
                verts.append(tuple(p))
                idx = len(verts) - 1
                cache[key] = idx
            return idx

        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_faces += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        faces = new_faces
    nodes = np.asarray(verts, dtype=np.float64) * radius
    tris = _orient_outward(nodes, np.asarray(faces, dtype=np.int64))
    return nodes, tris.astype(np.int32)


def geodesic_sphere(freq, radius=1.0):
    """Geodesic sphere of frequency ``freq``: every icosahedron face is cut
    into freq**2 triangles on a barycentric grid, then projected onto the
    sphere; 20 * freq**2 triangles in total (freq = 45 gives 40 500)."""
    v, f = _icosahedron()
    pts = []
    tri_local = []
    n = freq
    # local vertex index (i, j) with i + j <= n on each face
    loc = {}
    for i in range(n + 1):
        for j in range(n + 1 - i):
            loc[(i, j)] = len(loc)
    for i in range(n):
        for j in range(n - i):
            tri_local.append((loc[(i, j)], loc[(i + 1, j)], loc[(i, j + 1)]))
            if i + j + 1 < n:
                tri_local.append((loc[(i + 1, j)], loc[(i + 1, j + 1)], loc[(i, j + 1)]))
    tri_local = np.asarray(tri_local, dtype=np.int64)
    ij = np.array(list(loc.keys()), dtype=np.float64)
    all_tris = []
    for fi, (a, b, c) in enumerate(f):
        pa, pb, pc = v[a], v[b], v[c]
        w1 = ij[:, 0:1] / n
        w2 = ij[:, 1:2] / n
        p = pa * (1.0 - w1 - w2) + pb * w1 + pc * w2
        p /= np.linalg.norm(p, axis=1, keepdims=True)
        base = len(pts) * 0 + sum(len(x) for x in pts)
        pts.append(p)
        all_tris.append(tri_local + base)
    pts = np.concatenate(pts)
    tris = np.concatenate(all_tris)
    # merge vertices shared between faces (edges and corners)
    key = np.round(pts * 1e9).astype(np.int64)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    inv = inv.reshape(-1)
    order = np.argsort(first)
    remap = np.empty_like(order)
    remap[order] = np.arange(order.size)
    nodes = pts[first[order]] * radius
    tris = remap[inv[tris]]
    tris = _orient_outward(nodes, tris)
    return nodes, tris.astype(np.int32)


def _stereo_zoom(p, s):
    """Conformal self-map of the unit sphere that pulls points towards +x.

    Points are projected stereographically from the -x pole onto the plane
    x = 0 (w = (y + i z) / (1 + x)), scaled by 1/s and mapped back.  Near +x
    lengths shrink by 1/s, near -x they grow by s, so an initially uniform
    mesh becomes graded with a fine-to-coarse edge ratio of s**2 while
    every triangle keeps its angles."""
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    pole = 1.0 + x < 1e-12
    den = np.where(pole, 1.0, 1.0 + x)
    wy = y / den / s
    wz = z / den / s
    r2 = wy * wy + wz * wz
    out = np.empty_like(p)
    out[:, 0] = (1.0 - r2) / (1.0 + r2)
    out[:, 1] = 2.0 * wy / (1.0 + r2)
    out[:, 2] = 2.0 * wz / (1.0 + r2)
    # the projection pole is a fixed point of the map
    out[pole] = (-1.0, 0.0, 0.0)
    return out


def graded_ellipsoid_bump(freq=55, semi_axes=(0.075, 0.09, 0.11),
                          grading=5.0, bump_half=(0.010, 0.015),
                          bump_height=0.008):
    """Head-like ellipsoid with a raised-cosine bump on its +x side.

    A geodesic sphere (20 * freq**2 triangles) is graded conformally towards
    +x with a fine-to-coarse edge ratio ``grading``, scaled to the ellipsoid's
    semi-axes, and pushed outwards along the ellipsoid normal by
    ``bump_height * (1 + cos(pi * rho)) / 2`` where
    rho**2 = (y / bump_half[0])**2 + (z / bump_half[1])**2 < 1 and x > 0.
    Returns ``(nodes, tris, apex, apex_normal)``."""
    nodes, tris = geodesic_sphere(freq, 1.0)
    nodes = _stereo_zoom(nodes, grading ** 0.5)
    a = np.asarray(semi_axes, dtype=np.float64)
    e = nodes * a
    nrm = nodes / a
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    rho2 = (e[:, 1] / bump_half[0]) ** 2 + (e[:, 2] / bump_half[1]) ** 2
    inside = (rho2 < 1.0) & (e[:, 0] > 0)
    rho = np.sqrt(np.where(inside, rho2, 1.0))
    hgt = np.where(inside, bump_height * 0.5 * (1.0 + np.cos(np.pi * rho)), 0.0)
    e = e + nrm * hgt[:, None]
    apex = np.array([a[0] + bump_height, 0.0, 0.0])
    return e, tris, apex, np.array([1.0, 0.0, 0.0])


def box(lengths, h, origin=(0.0, 0.0, 0.0)):
    """Closed surface of the axis-aligned box [o, o + lengths] with a structured
    triangulation: each face cut into round(edge / h) (at least one) equal
    divisions per side, every rectangle split into two triangles along the
    same diagonal, vertices shared between faces, counter-clockwise seen from
    outside (normals out of the box)."""
    lx, ly, lz = (float(v) for v in lengths)
    o = np.asarray(origin, dtype=np.float64)
    n = [max(1, int(round(v / h))) for v in (lx, ly, lz)]
    index = {}
    nodes = []

    def node(i, j, k):
        key = (i, j, k)
        if key not in index:
            index[key] = len(nodes)
            nodes.append(o + np.array([lx * i / n[0], ly * j / n[1], lz * k / n[2]]))
        return index[key]

    tris = []
    # each face: the fixed axis, its side (0 or its division count), and the
    # two in-face axes ordered so that their cross product points outward
    faces = [(0, 0, 2, 1), (0, n[0], 1, 2), (1, 0, 0, 2), (1, n[1], 2, 0), (2, 0, 1, 0), (2, n[2], 0, 1)]
    for ax, side, u, v in faces:
        for a in range(n[u]):
            for b in range(n[v]):
                def at(da, db):
                    idx = [0, 0, 0]
                    idx[ax] = side
                    idx[u] = a + da
                    idx[v] = b + db
                    return node(*idx)
                p00, p10, p11, p01 = at(0, 0), at(1, 0), at(1, 1), at(0, 1)
                tris.append([p00, p10, p11])
                tris.append([p00, p11, p01])
    return np.array(nodes, dtype=np.float64), np.array(tris, dtype=np.int32)


def box_quads(lengths, h, origin=(0.0, 0.0, 0.0)):
    """The surface of box(lengths, h, origin) with every face rectangle kept
    whole: (n, 4) vertex indices, counter-clockwise seen from outside."""
    nodes, tris = box(lengths, h, origin)
    # box() emits each rectangle as (p00, p10, p11), (p00, p11, p01)
    t = tris.reshape(-1, 2, 3)
    quads = np.stack([t[:, 0, 0], t[:, 0, 1], t[:, 0, 2], t[:, 1, 2]], axis=1)
    return nodes, quads.astype(np.int32)


def uv_sphere(n_theta, n_phi, radius=1.0):
    """Latitude-longitude sphere: n_theta bands of equal polar angle, n_phi
    sectors.  Every cell between two latitude circles is a plane isosceles
    trapezoid (its four vertices are symmetric about the cell's mid meridian
    plane); the cells at the poles are triangles.  Elements: (n, 4) vertex
    indices, -1 in the last column of triangles, counter-clockwise seen from
    outside."""
    th = np.pi * np.arange(1, n_theta) / n_theta
    ph = 2.0 * np.pi * np.arange(n_phi) / n_phi
    nodes = [[0.0, 0.0, radius]]
    for t in th:
        for f in ph:
            nodes.append([radius * np.sin(t) * np.cos(f), radius * np.sin(t) * np.sin(f), radius * np.cos(t)])
    nodes.append([0.0, 0.0, -radius])
    south = len(nodes) - 1

    def ring(i, j):  # i-th latitude circle (0 = nearest the north pole)
        return 1 + i * n_phi + (j % n_phi)

    el = []
    for j in range(n_phi):
        el.append([0, ring(0, j), ring(0, j + 1), -1])
    for i in range(n_theta - 2):
        for j in range(n_phi):
            el.append([ring(i, j), ring(i + 1, j), ring(i + 1, j + 1), ring(i, j + 1)])
    for j in range(n_phi):
        el.append([south, ring(n_theta - 2, j + 1), ring(n_theta - 2, j), -1])
    return np.array(nodes, dtype=np.float64), np.array(el, dtype=np.int32)


def flat_patch(h=1.0):
    """Unit square in the z = 0 plane split into two triangles (normal +z)."""
    nodes = np.array([[0, 0, 0], [h, 0, 0], [h, h, 0], [0, h, 0]], dtype=np.float64)
    tris = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    return nodes, tris


def octahedron(radius=1.0):
    """Regular octahedron with 8 outward-oriented triangles."""
    nodes = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0],
                      [0, 0, 1], [0, 0, -1]], dtype=np.float64) * radius
    tris = np.array([[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4],
                     [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]], dtype=np.int64)
    return nodes, _orient_outward(nodes, tris).astype(np.int32)


def mean_edge_length(nodes, tris):
    """Mean length over the mesh's unique edges (used to pick a wavenumber
    for a target number of elements per wavelength)."""
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    e = np.sort(e, axis=1)
    e = np.unique(e, axis=0)
    return float(np.linalg.norm(nodes[e[:, 0]] - nodes[e[:, 1]], axis=1).mean())
