"""CPU pins of the oracle's coarse-mesh extraction and of neural normal mapping
onto mesh vertices (Sec. 5, the triangle-mesh example of Fig. 5).

  linear fields   the piecewise-linear surface of a linear field is exactly the
                  plane cut of the box: vertices on the plane, every triangle
                  facing along +grad, total area equal to the area of the
                  plane-box polygon computed from the box edges alone.
  sign patterns   all 256 corner patterns of one cube: vertex and triangle counts
                  from an independent enumeration of the six Kuhn tetrahedra, and
                  each triangle faces along the gradient of the linear
                  interpolant of the tetrahedron that holds it.
  closed shapes   sphere (genus 0), torus (genus 1), two spheres: every directed
                  edge has its reverse exactly once, the Euler characteristic is
                  2 - 2 genus per component, vertices inside the sphere by at most
                  the secant error bound, volume and area bracketed.
  normals         neural normal mapping onto points of an exact SDF is radial.
"""

import itertools

import numpy as np
import pytest

import nnm_inputs as ni
from oracle import mesh as M


def _grid(res, lo, hi):
    a = ni.grid_axis(res, lo, hi).astype(np.float64)
    z, y, x = np.meshgrid(a, a, a, indexing="ij")
    return x, y, z


def _tri_normals(V, Tr):
    p0, p1, p2 = V[Tr[:, 0]], V[Tr[:, 1]], V[Tr[:, 2]]
    return np.cross(p1 - p0, p2 - p0)


def _closed_and_euler(V, Tr):
    """Every directed edge appears once and its reverse once; returns V - E + F."""
    e = np.concatenate([Tr[:, [0, 1]], Tr[:, [1, 2]], Tr[:, [2, 0]]])
    key = e[:, 0].astype(np.int64) * len(V) + e[:, 1]
    rkey = e[:, 1].astype(np.int64) * len(V) + e[:, 0]
    assert len(np.unique(key)) == len(key), "a directed edge is used twice"
    assert np.array_equal(np.sort(key), np.sort(rkey)), "an edge lacks its reverse"
    n_edges = len(key) // 2
    used = np.unique(Tr)
    assert len(used) == len(V), "unreferenced vertices"
    return len(V) - n_edges + len(Tr)


def _signed_volume(V, Tr):
    p0, p1, p2 = V[Tr[:, 0]], V[Tr[:, 1]], V[Tr[:, 2]]
    return np.sum(np.einsum("ij,ij->i", p0, np.cross(p1, p2))) / 6.0


def _plane_box_area(g, c, lo, hi):
    """Area of {x in [lo,hi]^3 : g.x + c = 0} from the crossings of the 12 box edges."""
    pts = []
    corners = [np.array(p, np.float64) for p in itertools.product([lo, hi], repeat=3)]
    for a, b in itertools.combinations(corners, 2):
        if np.count_nonzero(a != b) != 1:
            continue
        fa, fb = g @ a + c, g @ b + c
        if (fa < 0) != (fb < 0):
            pts.append(a + fa / (fa - fb) * (b - a))
    pts = np.array(pts)
    n = g / np.linalg.norm(g)
    cen = pts.mean(0)
    u = pts[0] - cen
    u /= np.linalg.norm(u)
    w = np.cross(n, u)
    ang = np.arctan2((pts - cen) @ w, (pts - cen) @ u)
    P = pts[np.argsort(ang)]
    return 0.5 * abs(np.sum(np.cross(P, np.roll(P, -1, axis=0)) @ n))


@pytest.mark.parametrize("res", [2, 3, 5])
def test_linear_field_is_the_exact_plane_cut(res):
    rng = np.random.default_rng(100 + res)
    lo, hi = -1.0, 1.0
    x, y, z = _grid(res, lo, hi)
    for _ in range(20):
        g = rng.normal(size=3)
        g /= np.linalg.norm(g)
        c = rng.uniform(-0.5, 0.5)
        vals = (g[0] * x + g[1] * y + g[2] * z + c).astype(np.float32)
        V, Tr = M.marching_tets(vals, lo, hi)
        assert len(Tr) > 0
        # float32 rounding of the values moves vertices by ~1e-7
        assert np.max(np.abs(V @ g + c)) < 2e-6
        nrm = _tri_normals(V, Tr)
        area2 = np.linalg.norm(nrm, axis=1)
        big = area2 > 1e-9
        assert np.all(nrm[big] @ g / area2[big] > 1 - 1e-5), "triangle not facing along +grad"
        area = 0.5 * area2.sum()
        ref = _plane_box_area(g, c, lo, hi)
        assert abs(area - ref) <= 1e-5 * ref + 1e-7, (area, ref)


def _kuhn_tets():
    """The six tetrahedra of the unit cube: monotone corner paths 000 -> 111."""
    tets = []
    for perm in itertools.permutations(range(3)):
        p = np.zeros(3, int)
        corners = [p.copy()]
        for ax in perm:
            p[ax] = 1
            corners.append(p.copy())
        tets.append(np.array(corners))
    return tets


def test_all_corner_patterns_of_one_cube():
    rng = np.random.default_rng(7)
    tets = _kuhn_tets()
    edges = set()
    for T in tets:
        for a, b in itertools.combinations(range(4), 2):
            edges.add((tuple(T[a]), tuple(T[b])))
    assert len(edges) == 19
    for pattern in range(256):
        mag = rng.uniform(0.1, 1.0, size=8)
        vals = np.empty((2, 2, 2), np.float32)
        for corner in range(8):
            i, j, k = corner & 1, (corner >> 1) & 1, (corner >> 2) & 1
            vals[k, j, i] = -mag[corner] if (pattern >> corner) & 1 else mag[corner]
        V, Tr = M.marching_tets(vals, 0.0, 1.0)
        val_at = lambda p: float(vals[p[2], p[1], p[0]])
        inside = lambda p: val_at(p) < 0
        n_v = sum(inside(a) != inside(b) for a, b in edges)
        n_t = 0
        for T in tets:
            k_in = sum(inside(p) for p in T)
            n_t += {0: 0, 1: 1, 2: 2, 3: 1, 4: 0}[k_in]
        assert len(V) == n_v and len(Tr) == n_t, pattern
        if n_t == 0:
            continue
        nrm = _tri_normals(V, Tr)
        cen = V[Tr].mean(axis=1)
        for t in range(len(Tr)):
            if np.linalg.norm(nrm[t]) < 1e-12:
                continue
            found = False
            for T in tets:
                Q = T.astype(np.float64)
                A = (Q[1:] - Q[0]).T
                lam = np.linalg.solve(A, cen[t] - Q[0])
                if lam.min() < -1e-9 or lam.sum() > 1 + 1e-9:
                    continue
                f = np.array([val_at(p) for p in T], np.float64)
                grad = np.linalg.solve(A.T, f[1:] - f[0])
                assert nrm[t] @ grad > 0, (pattern, t)
                found = True
                break
            assert found, (pattern, t)


def _sdf_grid(res, lo, hi, fn):
    x, y, z = _grid(res, lo, hi)
    return fn(x, y, z).astype(np.float32)


@pytest.mark.parametrize("res", [17, 33])
def test_sphere_mesh_is_closed_genus0_and_bracketed(res):
    r = 0.6
    lo, hi = -1.0, 1.0
    V, Tr = M.marching_tets(_sdf_grid(res, lo, hi, lambda x, y, z: np.sqrt(x * x + y * y + z * z) - r), lo, hi)
    assert _closed_and_euler(V, Tr) == 2
    h = (hi - lo) / (res - 1)
    L = np.sqrt(3.0) * h  # longest grid edge (body diagonal)
    # secant of the convex |x| - r lies above it: vertices are inside by at most L^2 / (8 r')
    bound = L * L / (8 * (r - L)) + 1e-6
    rad = np.linalg.norm(V, axis=1)
    assert np.all(rad <= r + 1e-6) and np.all(r - rad <= bound), (rad.min(), bound)
    vol = _signed_volume(V, Tr)
    assert 4 / 3 * np.pi * (r - 2 * bound) ** 3 < vol < 4 / 3 * np.pi * r ** 3
    area = 0.5 * np.linalg.norm(_tri_normals(V, Tr), axis=1).sum()
    assert 4 * np.pi * (r - 2 * bound) ** 2 < area < 4 * np.pi * r ** 2


def test_torus_mesh_is_closed_genus1():
    R, r = 0.5, 0.2
    lo, hi = -1.0, 1.0
    fn = lambda x, y, z: np.sqrt((np.sqrt(x * x + y * y) - R) ** 2 + z * z) - r
    V, Tr = M.marching_tets(_sdf_grid(41, lo, hi, fn), lo, hi)
    assert _closed_and_euler(V, Tr) == 0
    vol = _signed_volume(V, Tr)
    assert abs(vol - 2 * np.pi ** 2 * R * r * r) < 0.05 * 2 * np.pi ** 2 * R * r * r


def test_two_spheres_two_components():
    lo, hi = -1.0, 1.0
    fn = lambda x, y, z: np.minimum(np.sqrt((x - 0.45) ** 2 + y * y + z * z),
                                    np.sqrt((x + 0.45) ** 2 + y * y + z * z)) - 0.3
    V, Tr = M.marching_tets(_sdf_grid(33, lo, hi, fn), lo, hi)
    assert _closed_and_euler(V, Tr) == 4


def test_empty_full_and_capacity():
    for fill in (1.0, -1.0):
        V, Tr = M.marching_tets(np.full((4, 4, 4), fill, np.float32), -1, 1)
        assert len(V) == 0 and len(Tr) == 0
    # NaN counts as outside: an inside node surrounded by NaN still closes
    vals = np.full((3, 3, 3), np.nan, np.float32)
    vals[1, 1, 1] = -1.0
    V, Tr = M.marching_tets(vals, -1, 1)
    assert len(Tr) > 0 and np.all(np.isnan(V))


def test_unit_normals_are_radial_on_an_exact_sdf():
    sc = ni.make_scene("stack3_512sq")
    for lvl in sc.levels:
        lvl.amplitude = 0.0
    rng = np.random.default_rng(3)
    x = rng.normal(size=(512, 3))
    x = (0.6 * x / np.linalg.norm(x, axis=1, keepdims=True) * rng.uniform(0.9, 1.1, (512, 1))).astype(np.float32)
    for level in range(len(sc.levels)):
        n = M.unit_normals(sc, level, x)
        x64 = x.astype(np.float64)
        np.testing.assert_allclose(n, x64 / np.linalg.norm(x64, axis=1, keepdims=True), atol=1e-14)
