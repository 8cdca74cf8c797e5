"""Closed triangle meshes used as cavity boundaries.

Every mesh is returned as ``(xyz, tri)`` with ``xyz`` a float64 ``(nv, 3)``
array and ``tri`` an int32 ``(nt, 3)`` array.  Triangles are ordered
counter-clockwise when seen from outside the closed surface, so the
right-hand normal ``(v1-v0) x (v2-v0)`` points away from the enclosed volume.
"""

import numpy as np

_PHI = (1.0 + 5.0 ** 0.5) / 2.0

# The 12 vertices of a regular icosahedron are the cyclic permutations of
# (0, +-1, +-phi).
_ICO_V = np.array(
    [(-1, _PHI, 0), (1, _PHI, 0), (-1, -_PHI, 0), (1, -_PHI, 0),
     (0, -1, _PHI), (0, 1, _PHI), (0, -1, -_PHI), (0, 1, -_PHI),
     (_PHI, 0, -1), (_PHI, 0, 1), (-_PHI, 0, -1), (-_PHI, 0, 1)],
    dtype=np.float64)


def _icosahedron_faces():
    """The 20 faces, found as the vertex triples at mutual edge length 2."""
    v = _ICO_V
    faces = []
    for i in range(12):
        for j in range(i + 1, 12):
            if abs(np.linalg.norm(v[i] - v[j]) - 2.0) > 1e-9:
                continue
            for k in range(j + 1, 12):
                if (abs(np.linalg.norm(v[i] - v[k]) - 2.0) < 1e-9
                        and abs(np.linalg.norm(v[j] - v[k]) - 2.0) < 1e-9):
                    faces.append((i, j, k))
    faces = np.array(faces, dtype=np.int64)
    assert faces.shape == (20, 3)
    return faces


def _orient_outward(xyz, tri, centre):
    """Flip triangles whose right-hand normal points towards ``centre``."""
    a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    g = np.cross(b - a, c - a)
    m = (a + b + c) / 3.0 - centre
    flip = np.einsum("ij,ij->i", g, m) < 0
    tri = tri.copy()
    tri[flip] = tri[flip][:, [0, 2, 1]]
    return tri


def icosphere(sub, radius=1.0, centre=(0.0, 0.0, 0.0)):
    """Unit icosahedron refined ``sub`` times (each triangle split into 4 at
    its edge midpoints, new vertices pushed onto the sphere), then scaled and
    translated.  ``sub`` refinements give ``20 * 4**sub`` triangles."""
    xyz = _ICO_V / np.linalg.norm(_ICO_V[0])
    tri = _orient_outward(xyz, _icosahedron_faces(), np.zeros(3))
    verts = [tuple(p) for p in xyz]
    for _ in range(int(sub)):
        cache = {}
        new_tri = []

        def mid(i, j):
            key = (min(i, j), max(i, j))
            if key not in cache:
                p = (np.asarray(verts[i]) + np.asarray(verts[j])) * 0.5
                p = p / np.linalg.norm(p)
                cache[key] = len(verts)
                verts.append(tuple(p))
            return cache[key]

        for a, b, c in tri:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_tri += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        tri = np.array(new_tri, dtype=np.int64)
    xyz = np.asarray(verts, dtype=np.float64) * float(radius)
    xyz = xyz + np.asarray(centre, dtype=np.float64)
    return xyz, tri.astype(np.int32)


def ellipsoid(sub, semi_axes, centre=(0.0, 0.0, 0.0)):
    """Icosphere vertices scaled along x, y, z by ``semi_axes``."""
    xyz, tri = icosphere(sub)
    xyz = xyz * np.asarray(semi_axes, dtype=np.float64)
    xyz = xyz + np.asarray(centre, dtype=np.float64)
    return xyz, tri


def merge_meshes(meshes):
    """Concatenate several ``(xyz, tri)`` meshes into one."""
    xs, ts, off = [], [], 0
    for xyz, tri in meshes:
        xs.append(xyz)
        ts.append(tri.astype(np.int64) + off)
        off += len(xyz)
    return np.concatenate(xs), np.concatenate(ts).astype(np.int32)


def random_cavity_centres(rng, count, box, min_dist, max_tries=100000):
    """Rejection-sample ``count`` centres uniformly in ``[-box/2, box/2]^3``
    with pairwise distance at least ``min_dist``."""
    out = []
    tries = 0
    while len(out) < count:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place cavities")
        c = rng.uniform(-box / 2.0, box / 2.0, size=3)
        if all(np.linalg.norm(c - o) >= min_dist for o in out):
            out.append(c)
    return np.array(out)


def box_mesh(lengths, divisions, origin=(0.0, 0.0, 0.0)):
    """Surface of the box origin + [0,Lx] x [0,Ly] x [0,Lz], each face cut
    into a structured grid of squares split into two triangles.

    ``divisions`` = (nx, ny, nz) cells along each axis.  Returns
    ``(xyz, tri, face)`` with ``face`` in 0..5 = (x=0, x=Lx, y=0, y=Ly, z=0,
    z=Lz); triangles are counter-clockwise seen from outside the box."""
    L = np.asarray(lengths, dtype=np.float64)
    n = [int(v) for v in divisions]
    o = np.asarray(origin, dtype=np.float64)
    verts = {}
    xyz = []

    def vid(p):
        key = tuple(np.round(p, 12))
        if key not in verts:
            verts[key] = len(xyz)
            xyz.append(p)
        return verts[key]

    tris, faces = [], []
    for axis in range(3):
        u, v = [a for a in range(3) if a != axis]
        for side in (0, 1):
            for i in range(n[u]):
                for j in range(n[v]):
                    corners = []
                    for di, dj in ((0, 0), (1, 0), (1, 1), (0, 1)):
                        p = np.zeros(3)
                        p[axis] = side * L[axis]
                        p[u] = (i + di) * L[u] / n[u]
                        p[v] = (j + dj) * L[v] / n[v]
                        corners.append(vid(o + p))
                    a, b, c, d = corners
                    for t in ((a, b, c), (a, c, d)):
                        tris.append(t)
                        faces.append(2 * axis + side)
    xyz = np.array(xyz)
    tri = np.array(tris, dtype=np.int64)
    # orient outward: the right-hand normal must point away from the centre
    tri = _orient_outward(xyz, tri, o + L / 2.0)
    return xyz, tri.astype(np.int32), np.array(faces, dtype=np.int32)
