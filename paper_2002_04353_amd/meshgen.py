"""Seeded synthetic P2-triangle meshes (input generation only).

This module produces the fixed computational meshes that both the GPU library
and the CPU oracle consume.  It holds none of the solver's arithmetic: no shape
functions, no element inverses, no owner map, no wall normals.  It only builds
point sets, triangulates them (scipy's Delaunay), attaches the six P2 nodes of
every triangle and records the topology (neighbours, periodic shifts, boundary
tags).

Mesh format (shared by both consumers, see ``include/alelb.h``):

``X``       float64 [N, 2]  computational node coordinates; for periodic meshes
            every node is canonical, inside [0, Lx) x [0, Ly).
``elem``    int32   [E, 6]  local order v0 v1 v2 m12 m20 m01: node 3+k is the
            mid-edge node of edge k, which lies opposite vertex k.  Triangles are
            counter-clockwise in their own frame.
``nbr``     int32   [E, 3]  element across edge k; -1 = wall, -2 = far field.
``pshift``  int8    [E, 3]  periodic shift code for crossing edge k (0 = none):
            code = (sx + 1) + 3 (sy + 1) - 4, and a point P in the frame of
            element e is P + (sx Lx, sy Ly) in the frame of nbr[e, k].
``period``  float64 [2]     (Lx, Ly), zeros for a non-periodic mesh.
``wall_edges`` int32 [W, 2] (element, local edge k) for every wall edge.

Frame of an element: vertex 0 sits at its canonical coordinates, every other
node at the periodic image nearest to vertex 0.  Elements are far smaller than
half a period, so this image is unique.

The computational mesh never moves (the paper maps the moving physical domain
onto a fixed computational one, Sec. II); the motion is an analytic map applied
by the solver.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.spatial import Delaunay

WALL = -1
FARFIELD = -2


@dataclass
class Mesh:
    X: np.ndarray
    elem: np.ndarray
    nbr: np.ndarray
    pshift: np.ndarray
    period: np.ndarray
    wall_edges: np.ndarray
    n_vertices: int
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.X.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.elem.shape[0])

    def arrays(self) -> dict:
        return dict(X=self.X, elem=self.elem, nbr=self.nbr, pshift=self.pshift,
                    period=self.period, wall_edges=self.wall_edges)

    def save(self, path: str) -> None:
        np.savez_compressed(path, n_vertices=self.n_vertices, **self.arrays())

    @staticmethod
    def load(path: str) -> "Mesh":
        z = np.load(path)  # plain arrays only, allow_pickle stays False
        return Mesh(X=z["X"], elem=z["elem"], nbr=z["nbr"], pshift=z["pshift"],
                    period=z["period"], wall_edges=z["wall_edges"],
                    n_vertices=int(z["n_vertices"]))


def shift_code(sx: np.ndarray, sy: np.ndarray) -> np.ndarray:
    return ((sx + 1) + 3 * (sy + 1) - 4).astype(np.int8)


def _min_image(p: np.ndarray, ref: np.ndarray, period: np.ndarray) -> np.ndarray:
    """Image of p nearest to ref (componentwise; period 0 = not periodic)."""
    out = p.copy()
    for d in range(2):
        if period[d] > 0:
            out[..., d] = p[..., d] + period[d] * np.round((ref[..., d] - p[..., d]) / period[d])
    return out


def _attach_p2(Xv: np.ndarray, tris: np.ndarray, period: np.ndarray,
               boundary_tag) -> Mesh:
    """Add mid-edge nodes, neighbours and periodic shifts to a triangulation.

    Xv: canonical vertex coordinates [V, 2]; tris: vertex ids [E, 3].  The
    orientation is fixed here so that every triangle is counter-clockwise in
    its own frame.  ``boundary_tag(a, b)`` returns WALL or FARFIELD for a
    boundary edge between vertices a and b.
    """
    V = Xv.shape[0]
    E = tris.shape[0]
    tris = tris.astype(np.int64).copy()
    # frame positions of the three vertices
    p0 = Xv[tris[:, 0]]
    p1 = _min_image(Xv[tris[:, 1]], p0, period)
    p2 = _min_image(Xv[tris[:, 2]], p0, period)
    cross = (p1[:, 0] - p0[:, 0]) * (p2[:, 1] - p0[:, 1]) - (p1[:, 1] - p0[:, 1]) * (p2[:, 0] - p0[:, 0])
    flip = cross < 0
    tris[flip, 1], tris[flip, 2] = tris[flip, 2].copy(), tris[flip, 1].copy()
    p1, p2 = np.where(flip[:, None], p2, p1), np.where(flip[:, None], p1, p2)
    fp = np.stack([p0, p1, p2], axis=1)  # [E, 3, 2] vertex positions in each frame

    # edge k joins vertices k+1 and k+2
    ea = np.stack([tris[:, 1], tris[:, 2], tris[:, 0]], axis=1)  # [E,3]
    eb = np.stack([tris[:, 2], tris[:, 0], tris[:, 1]], axis=1)
    pa = np.stack([fp[:, 1], fp[:, 2], fp[:, 0]], axis=1)  # [E,3,2]
    pb = np.stack([fp[:, 2], fp[:, 0], fp[:, 1]], axis=1)
    lo = np.minimum(ea, eb)
    hi = np.maximum(ea, eb)
    plo = np.where((ea <= eb)[..., None], pa, pb)
    phi = np.where((ea <= eb)[..., None], pb, pa)
    dvec = phi - plo
    dcan = Xv[hi] - Xv[lo]
    img = np.zeros(lo.shape + (2,), dtype=np.int64)
    for d in range(2):
        if period[d] > 0:
            img[..., d] = np.round((dvec[..., d] - dcan[..., d]) / period[d]).astype(np.int64)
    key = np.stack([lo, hi, img[..., 0], img[..., 1]], axis=-1).reshape(-1, 4)
    uniq, inv, counts = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    inv = inv.reshape(E, 3)
    if np.any(counts > 2):
        raise ValueError("non-manifold triangulation: an edge has more than two triangles")
    n_edges = uniq.shape[0]
    # mid-node coordinates (canonical)
    first = np.full(n_edges, -1, dtype=np.int64)
    flat = np.arange(E * 3)
    first[inv.reshape(-1)[::-1]] = flat[::-1]
    fe, fk = first // 3, first % 3
    mid = 0.5 * (pa[fe, fk] + pb[fe, fk])
    for d in range(2):
        if period[d] > 0:
            mid[:, d] = np.mod(mid[:, d], period[d])
            mid[:, d] = np.where(mid[:, d] >= period[d], mid[:, d] - period[d], mid[:, d])
    X = np.concatenate([Xv, mid], axis=0)
    elem = np.concatenate([tris, V + inv], axis=1).astype(np.int32)

    # neighbours: the other (element, edge) owning the same edge id
    owners = np.full((n_edges, 2), -1, dtype=np.int64)
    slot_e = flat // 3
    order = np.argsort(inv.reshape(-1), kind="stable")
    sorted_ids = inv.reshape(-1)[order]
    starts = np.searchsorted(sorted_ids, np.arange(n_edges))
    owners[:, 0] = order[starts]
    two = counts == 2
    owners[two, 1] = order[starts[two] + 1]
    nbr = np.empty((E, 3), dtype=np.int32)
    pshift = np.zeros((E, 3), dtype=np.int8)
    eid = inv.reshape(-1)
    me = flat
    o0, o1 = owners[eid, 0], owners[eid, 1]
    other = np.where(o0 == me, o1, o0)
    nb = np.where(other >= 0, other // 3, -1)
    nbr_flat = nb.copy()
    bidx = np.nonzero(nb < 0)[0]
    for j in bidx:
        e, k = divmod(int(j), 3)
        nbr_flat[j] = boundary_tag(int(ea[e, k]), int(eb[e, k]))
    nbr[:] = nbr_flat.reshape(E, 3)
    # periodic shift for crossing into the neighbour's frame
    if np.any(period > 0):
        inner = np.nonzero(nb >= 0)[0]
        e_in, k_in = inner // 3, inner % 3
        n_in = nb[inner]
        # position of vertex ea (edge start) in my frame and in the neighbour's frame
        pe = pa[e_in, k_in]
        anchor_n = Xv[tris[n_in, 0]]
        pn = _min_image(Xv[ea[e_in, k_in]], anchor_n, period)
        s = np.zeros((inner.size, 2), dtype=np.int64)
        for d in range(2):
            if period[d] > 0:
                s[:, d] = np.round((pn[:, d] - pe[:, d]) / period[d]).astype(np.int64)
        codes = shift_code(s[:, 0], s[:, 1])
        ps = pshift.reshape(-1)
        ps[inner] = codes
        pshift = ps.reshape(E, 3)
    walls = np.argwhere(nbr == WALL).astype(np.int32)
    return Mesh(X=X.astype(np.float64), elem=elem, nbr=nbr, pshift=pshift,
                period=np.asarray(period, dtype=np.float64), wall_edges=walls,
                n_vertices=V)


def _attach_q2(Xv: np.ndarray, quads: np.ndarray, period: np.ndarray, boundary_tag) -> Mesh:
    """9-node Lagrange quadrilaterals (the element of Sec. III) from a quad mesh.

    Xv: canonical vertex coordinates [V, 2]; quads: vertex ids [E, 4].  Each
    quad is made counter-clockwise in its own frame.  Local nodes: corners
    0..3, then node 4+k at the midpoint of edge k (corner k to corner k+1),
    then the centre (node 8); edge and centre nodes sit where the bilinear
    map of the corners puts (0, -1), (1, 0), (0, 1), (-1, 0) and (0, 0).
    Edge k is crossed into nbr[e, k]; ``boundary_tag(a, b)`` gives WALL or
    FARFIELD for a boundary edge between vertices a and b.
    """
    V = Xv.shape[0]
    E = quads.shape[0]
    q = quads.astype(np.int64).copy()
    p0 = Xv[q[:, 0]]
    fp = np.stack([p0] + [_min_image(Xv[q[:, k]], p0, period) for k in (1, 2, 3)], axis=1)  # [E,4,2]
    area2 = np.zeros(E)
    for k in range(4):
        a, b = fp[:, k], fp[:, (k + 1) % 4]
        area2 += a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0]
    flip = area2 < 0
    q[flip] = q[flip][:, [0, 3, 2, 1]]
    fp[flip] = fp[flip][:, [0, 3, 2, 1]]
    ea = q
    eb = np.roll(q, -1, axis=1)
    pa = fp
    pb = np.roll(fp, -1, axis=1)
    lo, hi = np.minimum(ea, eb), np.maximum(ea, eb)
    plo = np.where((ea <= eb)[..., None], pa, pb)
    phi = np.where((ea <= eb)[..., None], pb, pa)
    dvec, dcan = phi - plo, Xv[hi] - Xv[lo]
    img = np.zeros(lo.shape + (2,), dtype=np.int64)
    for d in range(2):
        if period[d] > 0:
            img[..., d] = np.round((dvec[..., d] - dcan[..., d]) / period[d]).astype(np.int64)
    key = np.stack([lo, hi, img[..., 0], img[..., 1]], axis=-1).reshape(-1, 4)
    uniq, inv, counts = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    inv = inv.reshape(E, 4)
    if np.any(counts > 2):
        raise ValueError("non-manifold quad mesh: an edge has more than two quads")
    n_edges = uniq.shape[0]
    flat = np.arange(E * 4)
    first = np.full(n_edges, -1, dtype=np.int64)
    first[inv.reshape(-1)[::-1]] = flat[::-1]
    fe, fk = first // 4, first % 4
    mid = 0.5 * (pa[fe, fk] + pb[fe, fk])
    cen = fp.mean(axis=1)
    for arr in (mid, cen):
        for d in range(2):
            if period[d] > 0:
                arr[:, d] = np.mod(arr[:, d], period[d])
                arr[:, d] = np.where(arr[:, d] >= period[d], arr[:, d] - period[d], arr[:, d])
    X = np.concatenate([Xv, mid, cen], axis=0)
    elem = np.concatenate([q, V + inv, (V + n_edges + np.arange(E))[:, None]], axis=1).astype(np.int32)
    order = np.argsort(inv.reshape(-1), kind="stable")
    sorted_ids = inv.reshape(-1)[order]
    starts = np.searchsorted(sorted_ids, np.arange(n_edges))
    owners = np.full((n_edges, 2), -1, dtype=np.int64)
    owners[:, 0] = order[starts]
    two = counts == 2
    owners[two, 1] = order[starts[two] + 1]
    eid = inv.reshape(-1)
    o0, o1 = owners[eid, 0], owners[eid, 1]
    other = np.where(o0 == flat, o1, o0)
    nb = np.where(other >= 0, other // 4, -1)
    nbr_flat = nb.copy()
    for j in np.nonzero(nb < 0)[0]:
        e, k = divmod(int(j), 4)
        nbr_flat[j] = boundary_tag(int(ea[e, k]), int(eb[e, k]))
    nbr = nbr_flat.reshape(E, 4).astype(np.int32)
    pshift = np.zeros((E, 4), dtype=np.int8)
    if np.any(period > 0):
        inner = np.nonzero(nb >= 0)[0]
        e_in, k_in = inner // 4, inner % 4
        n_in = nb[inner]
        pe = pa[e_in, k_in]
        anchor_n = Xv[q[n_in, 0]]
        pn = _min_image(Xv[ea[e_in, k_in]], anchor_n, period)
        sft = np.zeros((inner.size, 2), dtype=np.int64)
        for d in range(2):
            if period[d] > 0:
                sft[:, d] = np.round((pn[:, d] - pe[:, d]) / period[d]).astype(np.int64)
        ps = pshift.reshape(-1)
        ps[inner] = shift_code(sft[:, 0], sft[:, 1])
        pshift = ps.reshape(E, 4)
    walls = np.argwhere(nbr == WALL).astype(np.int32)
    return Mesh(X=X.astype(np.float64), elem=elem, nbr=nbr, pshift=pshift,
                period=np.asarray(period, dtype=np.float64), wall_edges=walls, n_vertices=V)


def quad_convexity(m: Mesh) -> float:
    """Smallest corner cross product over all quads, relative to the squared
    mean edge length (> 0: every quad is strictly convex)."""
    fp = np.stack([m.X[m.elem[:, 0]]] + [_min_image(m.X[m.elem[:, k]], m.X[m.elem[:, 0]], m.period)
                                        for k in (1, 2, 3)], axis=1)
    worst = np.inf
    for k in range(4):
        a, b, c = fp[:, (k - 1) % 4], fp[:, k], fp[:, (k + 1) % 4]
        cr = (b[:, 0] - a[:, 0]) * (c[:, 1] - b[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - b[:, 0])
        l2 = np.sum((c - b) ** 2, axis=1) + np.sum((b - a) ** 2, axis=1)
        worst = min(worst, float(np.min(cr / (0.5 * l2))))
    return worst


def periodic_square_quads(nx: int, ny: int, Lx: float = 1.0, Ly: float = 1.0, jitter: float = 0.2,
                          seed: int = 1) -> Mesh:
    """Torus Q2 mesh on [0,Lx) x [0,Ly): an nx-by-ny grid of vertices, each moved
    by +-``jitter`` spacings, joined into quads (i, j) (i+1, j) (i+1, j+1)
    (i, j+1).  N = 4 V nodes (V vertices, 2 V edge nodes, V centres)."""
    if not 0 <= jitter < 0.5:
        raise ValueError("jitter must lie in [0, 0.5) to keep the quads convex")
    rng = np.random.default_rng(seed)
    hx, hy = Lx / nx, Ly / ny
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    px = (ii.reshape(-1) + 0.5 + rng.uniform(-jitter, jitter, nx * ny)) * hx
    py = (jj.reshape(-1) + 0.5 + rng.uniform(-jitter, jitter, nx * ny)) * hy
    Xv = np.stack([px, py], axis=1)
    vid = lambda i, j: (j % ny) * nx + (i % nx)  # noqa: E731
    quads = np.array([[vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)]
                      for j in range(ny) for i in range(nx)], dtype=np.int64)

    def no_boundary(a, b):
        raise ValueError("periodic mesh has a boundary edge")

    m = _attach_q2(Xv, quads, np.array([Lx, Ly]), no_boundary)
    m.meta.update(kind="periodic_square_quads", nx=nx, ny=ny, Lx=Lx, Ly=Ly, jitter=jitter, seed=seed)
    return m


def structured_square_quads(nx: int, ny: int, Lx: float = 1.0, Ly: float = 1.0, jitter: float = 0.0,
                            seed: int = 0, tag=FARFIELD) -> Mesh:
    """Non-periodic Q2 mesh of [0,Lx] x [0,Ly] (small test meshes): an
    (nx+1)-by-(ny+1) grid of vertices, interior ones moved by +-jitter
    spacings, joined into nx*ny quads.  Every boundary edge gets ``tag``."""
    if not 0 <= jitter < 0.5:
        raise ValueError("jitter must lie in [0, 0.5) to keep the quads convex")
    rng = np.random.default_rng(seed)
    xs = np.linspace(0.0, Lx, nx + 1)
    ys = np.linspace(0.0, Ly, ny + 1)
    P = np.stack(np.meshgrid(xs, ys, indexing="xy"), axis=-1).reshape(-1, 2)
    inner = (P[:, 0] > 0) & (P[:, 0] < Lx) & (P[:, 1] > 0) & (P[:, 1] < Ly)
    J = rng.uniform(-jitter, jitter, P.shape) * np.array([Lx / nx, Ly / ny])
    P[inner] += J[inner]
    vid = lambda i, j: j * (nx + 1) + i  # noqa: E731
    quads = np.array([[vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)]
                      for j in range(ny) for i in range(nx)], dtype=np.int64)
    m = _attach_q2(P, quads, np.zeros(2), lambda a, b: tag)
    m.meta.update(kind="square_quads", nx=nx, ny=ny, Lx=Lx, Ly=Ly)
    return m


def _open_te_polygon(chord: float, spacing: float, n_base: int, t: float = 0.12):
    """Counter-clockwise surface polygon of the open-trailing-edge NACA 4-digit
    section (last coefficient -0.1015: a blunt base of 0.00252 chord): upper
    surface from the upper base corner to the leading edge, lower surface to
    the lower base corner, then n_base - 1 points along the base.  Returns
    (points, index of the lower base corner)."""
    s = np.linspace(0.0, math.pi, 20001)
    xd = 0.5 * (1.0 - np.cos(s))
    yd = 5.0 * t * (0.2969 * np.sqrt(xd) - 0.1260 * xd - 0.3516 * xd**2 + 0.2843 * xd**3 - 0.1015 * xd**4)
    out = []
    for curve in (np.stack([xd[::-1], yd[::-1]], axis=1), np.stack([xd, -yd], axis=1)):
        c = curve * chord
        seg = np.linalg.norm(np.diff(c, axis=0), axis=1)
        arc = np.concatenate([[0.0], np.cumsum(seg)])
        n = max(2, int(round(arc[-1] / spacing)))
        ss = np.linspace(0.0, arc[-1], n + 1)[:-1]
        out.append(np.stack([np.interp(ss, arc, c[:, 0]), np.interp(ss, arc, c[:, 1])], axis=1))
    lo = c[-1]
    up = out[0][0]
    out[1] = np.concatenate([out[1], lo[None]], axis=0)
    f = np.arange(1, n_base)[:, None] / n_base
    out.append(lo[None] + f * (up - lo)[None])
    poly = np.concatenate(out, axis=0)
    return poly, out[0].shape[0] + out[1].shape[0] - 1


def _inside_polygon(pts: np.ndarray, poly: np.ndarray) -> np.ndarray:
    """Even-odd point-in-polygon test."""
    inside = np.zeros(pts.shape[0], dtype=bool)
    a = poly
    b = np.roll(poly, -1, axis=0)
    for (ax, ay), (bx, by) in zip(a, b):
        cond = (ay > pts[:, 1]) != (by > pts[:, 1])
        xint = ax + (pts[:, 1] - ay) * (bx - ax) / np.where(by != ay, by - ay, 1.0)
        inside ^= cond & (pts[:, 0] < xint)
    return inside


def naca_omesh_quads(n_nodes_target: int = 200_000, chord: float = 200.0, radius_c: float = 20.0,
                     first: float = 0.5, growth: float = 1.1, surface_ratio: float = 1.4,
                     structured_layers: int = 4, n_base: int = 1, jitter: float = 0.2,
                     seed: int = 3) -> Mesh:
    """Seeded NACA0012 mesh of 9-node quadrilaterals: orthogonal structured
    layers at the wall, unstructured quadrilaterals elsewhere (the layout of
    the paper's airfoil meshes, Sec. V.B).

    Built on a coarse mesh at twice the final spacing, then refined into
    quadrilaterals: every coarse structured quad splits into 4 (edge midpoints
    and centre), every coarse triangle into 3 (edge midpoints and centroid);
    the splits agree on shared edges, so the result is conforming.  Final
    sizes: first layer ``first``, surface spacing surface_ratio * first.
    The section has the open trailing edge of the 4-digit formula: a blunt
    base of n_base coarse wall edges, whose near-wall rays fan from one base
    corner's bisector to the other's, so no quad has a corner near 180
    degrees (an O-type layer around a sharp trailing edge would, and the
    solver diverges there).  Keep n_base small: base cells much narrower than
    the first layer make the correction term, a second derivative, stiff
    (with 4 coarse base edges the pitching case diverged within 10 steps).  Structured
    coarse layers: ``structured_layers`` normal offsets, heights first*2,
    growing by ``growth``.  Beyond them, jittered offset curves as in
    ``naca_omesh`` (spacing s0 + g d, g set for the node count), Delaunay.
    """
    rng = np.random.default_rng(seed)
    f_c = 2.0 * first
    s0_c = 2.0 * surface_ratio * first
    poly, i_lo = _open_te_polygon(chord, s0_c, n_base)
    ns = poly.shape[0]
    i_up = 0
    # ray directions: averaged outward edge normals; across the base a fan
    e = np.roll(poly, -1, axis=0) - poly
    en = np.stack([e[:, 1], -e[:, 0]], axis=1)
    en /= np.linalg.norm(en, axis=1)[:, None]
    nv = en + np.roll(en, 1, axis=0)
    nv /= np.linalg.norm(nv, axis=1)[:, None]
    a_lo = math.atan2(nv[i_lo, 1], nv[i_lo, 0])
    a_up = math.atan2(nv[i_up, 1], nv[i_up, 0])
    for j in range(1, n_base):
        a = a_lo + (a_up - a_lo) * j / n_base
        nv[i_lo + j] = [math.cos(a), math.sin(a)]
    dl = [0.0]
    for j in range(structured_layers):
        dl.append(dl[-1] + f_c * growth**j)
    rings = [poly + d * nv for d in dl]
    d_s = dl[-1]
    step_s = f_c * growth ** (structured_layers - 1)
    # outer layers: offset curves at d_s + ..., spacing s0 + g d (coarse), g by bisection
    d_max = radius_c * chord - 0.5 * chord
    Vs = ns * len(rings)
    v_target = n_nodes_target / 24.0

    def plan(g):
        ds = [d_s]
        j = 0
        while ds[-1] < d_max:
            d = ds[-1]
            ht = s0_c + g * d
            st = min(step_s * growth ** (j + 1), ht)
            ds.append(min(d + st, d_max) if d_max - (d + st) > 0.5 * st else d_max)
            j += 1
        return np.asarray(ds[1:])

    def count(g):
        ds = plan(g)
        return Vs + float(np.sum((2.03 * chord + 2 * math.pi * ds) / (s0_c + g * ds)))

    lo_g, hi_g = 1e-4, 16.0
    for _ in range(60):
        mid_g = math.sqrt(lo_g * hi_g)
        if count(mid_g) > v_target:
            lo_g = mid_g
        else:
            hi_g = mid_g
    g = math.sqrt(lo_g * hi_g)
    ds = plan(g)
    body, _ = _open_te_polygon(chord, 0.25 * s0_c, n_base)
    outer = []
    for j, d in enumerate(ds):
        ht = s0_c + g * d
        cur = _offset_curve(body, d, dphi=min(0.04, 0.25 * ht / max(d, 1e-9)))
        pts = _resample_closed(cur, ht, rng.uniform(0.0, 1.0))
        if j < len(ds) - 1:
            step = ds[j] - (ds[j - 1] if j else d_s)
            amp = jitter * min(ht, step)
            pts = pts + rng.uniform(-amp, amp, pts.shape)
        outer.append(pts)
    ring = rings[-1]
    Xo = np.concatenate(outer, axis=0)
    Xo = Xo[~_inside_polygon(Xo, ring)]
    n_outer = outer[-1].shape[0]
    Xc = np.concatenate(rings + [Xo], axis=0)
    r0 = ns * (len(rings) - 1)  # first id of the last ring
    sub = np.concatenate([np.arange(r0, r0 + ns), ns * len(rings) + np.arange(Xo.shape[0])])
    tri = sub[Delaunay(Xc[sub]).simplices.astype(np.int64)]
    on_ring = np.all(tri < r0 + ns, axis=1)
    cen = Xc[tri].mean(axis=1)
    drop = np.zeros(tri.shape[0], dtype=bool)
    drop[on_ring] = _inside_polygon(cen[on_ring], ring)
    tri = tri[~drop]
    edges = set()
    for k in range(3):
        a_, b_ = tri[:, (k + 1) % 3], tri[:, (k + 2) % 3]
        edges.update(zip(np.minimum(a_, b_).tolist(), np.maximum(a_, b_).tolist()))
    for i in range(ns):
        u, v = r0 + i, r0 + (i + 1) % ns
        if (min(u, v), max(u, v)) not in edges:
            raise ValueError(f"structured ring edge {i} is not a Delaunay edge; use more outer spacing")
    # refine into quadrilaterals: coarse vertices, then one node per coarse edge, then per cell
    Vc = Xc.shape[0]
    cells_q = np.array([[j * ns + i, j * ns + (i + 1) % ns, (j + 1) * ns + (i + 1) % ns, (j + 1) * ns + i]
                        for j in range(len(rings) - 1) for i in range(ns)], dtype=np.int64)
    ce = [np.stack([cells_q[:, k], cells_q[:, (k + 1) % 4]], axis=1) for k in range(4)]
    te = [np.stack([tri[:, k], tri[:, (k + 1) % 3]], axis=1) for k in range(3)]
    alle = np.concatenate(ce + te, axis=0)
    key = np.sort(alle, axis=1)
    uniq, inv = np.unique(key, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    nq, nt_ = cells_q.shape[0], tri.shape[0]
    mid_q = [Vc + inv[k * nq:(k + 1) * nq] for k in range(4)]
    off = 4 * nq
    mid_t = [Vc + inv[off + k * nt_: off + (k + 1) * nt_] for k in range(3)]
    Xm = 0.5 * (Xc[uniq[:, 0]] + Xc[uniq[:, 1]])
    c_q = Vc + uniq.shape[0] + np.arange(nq)
    c_t = Vc + uniq.shape[0] + nq + np.arange(nt_)
    Xf = np.concatenate([Xc, Xm, Xc[cells_q].mean(axis=1), Xc[tri].mean(axis=1)], axis=0)
    quads = []
    for k in range(4):  # the sub-quad at corner k: corner, next edge node, centre, previous edge node
        quads.append(np.stack([cells_q[:, k], mid_q[k], c_q, mid_q[(k - 1) % 4]], axis=1))
    for k in range(3):
        quads.append(np.stack([tri[:, k], mid_t[k], c_t, mid_t[(k - 1) % 3]], axis=1))
    quads = np.concatenate(quads, axis=0)
    surf = np.zeros(Xf.shape[0], dtype=bool)
    surf[:ns] = True
    wall_e = np.all(uniq < ns, axis=1) & (((uniq[:, 1] - uniq[:, 0]) == 1) | ((uniq[:, 0] == 0) & (uniq[:, 1] == ns - 1)))
    surf[Vc + np.nonzero(wall_e)[0]] = True
    far = np.zeros(Xf.shape[0], dtype=bool)
    far[Vc - n_outer:Vc] = True
    far_e = np.all(uniq >= Vc - n_outer, axis=1)
    far[Vc + np.nonzero(far_e)[0]] = True

    def tag(a, b):
        if surf[a] and surf[b]:
            return WALL
        if far[a] and far[b]:
            return FARFIELD
        raise ValueError(f"unexpected boundary edge {a}-{b}")

    m = _attach_q2(Xf, quads, np.zeros(2), tag)
    if m.wall_edges.shape[0] != 2 * ns:
        raise ValueError("wall edge count differs from twice the coarse surface point count")
    if quad_convexity(m) <= 0.0:
        raise ValueError("a quadrilateral is not strictly convex")
    m.meta.update(kind="naca_omesh_quads", chord=chord, radius_c=radius_c, first=first, growth=growth,
                  s0=surface_ratio * first, g=0.5 * g, structured_layers=2 * structured_layers,
                  n_surface=2 * ns, n_base=n_base, seed=seed)
    return m


# ---------------------------------------------------------------------------
# periodic jittered Delaunay meshes (uniform-flow and vortex workloads)
# ---------------------------------------------------------------------------

def periodic_square(nx: int, ny: int, Lx: float = 1.0, Ly: float = 1.0,
                    jitter: float = 0.25, seed: int = 1) -> Mesh:
    """Torus P2 mesh on [0,Lx) x [0,Ly): an nx-by-ny grid of vertices, each moved
    by a uniform jitter of +-``jitter`` grid spacings, triangulated by Delaunay
    on a 3x3 tiling; the copy of each triangle whose centroid falls in the
    central tile is kept.  N = 4 V and E = 2 V on the torus.
    """
    if jitter <= 0:
        raise ValueError("jitter must be positive (ties make the periodic Delaunay ambiguous)")
    rng = np.random.default_rng(seed)
    hx, hy = Lx / nx, Ly / ny
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    px = (ii.reshape(-1) + 0.5 + rng.uniform(-jitter, jitter, nx * ny)) * hx
    py = (jj.reshape(-1) + 0.5 + rng.uniform(-jitter, jitter, nx * ny)) * hy
    Xv = np.stack([px, py], axis=1)
    V = Xv.shape[0]
    tiles = []
    for sy in (-1, 0, 1):
        for sx in (-1, 0, 1):
            tiles.append(Xv + np.array([sx * Lx, sy * Ly]))
    P = np.concatenate(tiles, axis=0)
    tri = Delaunay(P).simplices
    cen = P[tri].mean(axis=1)
    keep = (cen[:, 0] >= 0) & (cen[:, 0] < Lx) & (cen[:, 1] >= 0) & (cen[:, 1] < Ly)
    tris = tri[keep] % V
    if tris.shape[0] != 2 * V:
        raise ValueError(f"periodic triangulation has {tris.shape[0]} triangles, expected {2 * V}")

    def no_boundary(a, b):
        raise ValueError("periodic mesh has a boundary edge")

    m = _attach_p2(Xv, tris, np.array([Lx, Ly]), no_boundary)
    if m.n_nodes != 4 * V:
        raise ValueError("periodic P2 mesh must have N = 4 V nodes")
    m.meta.update(kind="periodic_square", nx=nx, ny=ny, Lx=Lx, Ly=Ly, jitter=jitter, seed=seed)
    return m


# ---------------------------------------------------------------------------
# NACA0012 O-mesh (airfoil workloads)
# ---------------------------------------------------------------------------

def naca00xx_thickness(x: np.ndarray, t: float = 0.12) -> np.ndarray:
    """Half thickness of a symmetric 4-digit NACA section at x in [0, 1] (unit
    chord), closed-trailing-edge form of the last coefficient."""
    return 5.0 * t * (0.2969 * np.sqrt(x) - 0.1260 * x - 0.3516 * x**2
                      + 0.2843 * x**3 - 0.1036 * x**4)


def _airfoil_polygon(chord: float, spacing: float, t: float = 0.12) -> np.ndarray:
    """Closed counter-clockwise surface polygon (trailing edge first, no repeat)
    with nearly uniform arc-length spacing."""
    # dense cosine-spaced polyline, upper surface TE -> LE, lower surface LE -> TE
    s = np.linspace(0.0, math.pi, 20001)
    xd = 0.5 * (1.0 - np.cos(s))
    yd = naca00xx_thickness(xd, t)
    upper = np.stack([xd[::-1], yd[::-1]], axis=1)  # TE -> LE
    lower = np.stack([xd[1:], -yd[1:]], axis=1)     # LE -> TE
    dense = np.concatenate([upper, lower[:-1]], axis=0) * chord
    closed = np.concatenate([dense, dense[:1]], axis=0)
    seg = np.linalg.norm(np.diff(closed, axis=0), axis=1)
    arc = np.concatenate([[0.0], np.cumsum(seg)])
    per = arc[-1]
    # keep the leading edge as a sample: resample each half separately
    i_le = upper.shape[0] - 1
    out = []
    for a0, a1 in ((arc[0], arc[i_le]), (arc[i_le], per)):
        n = max(2, int(round((a1 - a0) / spacing)))
        ss = np.linspace(a0, a1, n + 1)[:-1]
        out.append(np.stack([np.interp(ss, arc, closed[:, 0]),
                             np.interp(ss, arc, closed[:, 1])], axis=1))
    poly = np.concatenate(out, axis=0)
    return poly


def _offset_curve(poly: np.ndarray, d: float, dphi: float = 0.04) -> np.ndarray:
    """Boundary of {x : dist(x, convex polygon) <= d}, densely sampled (closed,
    counter-clockwise, no repeat): edges shifted along their outward normal and
    circular arcs around the vertices."""
    n = poly.shape[0]
    nxt = np.roll(poly, -1, axis=0)
    e = nxt - poly
    en = np.stack([e[:, 1], -e[:, 0]], axis=1)  # outward normal for a CCW polygon
    en /= np.linalg.norm(en, axis=1)[:, None]
    ang = np.arctan2(en[:, 1], en[:, 0])
    pts = []
    for i in range(n):
        a_in = ang[i - 1]
        a_out = ang[i]
        da = (a_out - a_in) % (2 * math.pi)
        if da > math.pi:  # not convex at this vertex: no arc
            da = 0.0
        m = max(1, int(math.ceil(da / dphi)))
        for j in range(m + 1):
            a = a_in + da * j / m
            pts.append(poly[i] + d * np.array([math.cos(a), math.sin(a)]))
    return np.asarray(pts)


def _resample_closed(curve: np.ndarray, h: float, phase: float) -> np.ndarray:
    closed = np.concatenate([curve, curve[:1]], axis=0)
    seg = np.linalg.norm(np.diff(closed, axis=0), axis=1)
    arc = np.concatenate([[0.0], np.cumsum(seg)])
    per = arc[-1]
    n = max(64, int(round(per / h)))
    ss = (np.arange(n) + phase) * (per / n)
    return np.stack([np.interp(ss, arc, closed[:, 0]), np.interp(ss, arc, closed[:, 1])], axis=1)


def _layer_plan(chord, first, growth, s0, g, d_max):
    ds = [0.0]
    j = 0
    while ds[-1] < d_max:
        d = ds[-1]
        ht = s0 + g * d
        step = min(first * growth**j, ht)
        ds.append(min(d + step, d_max) if d_max - (d + step) > 0.5 * step else d_max)
        j += 1
    return np.asarray(ds)


def _estimate_vertices(chord, first, growth, s0, g, d_max):
    ds = _layer_plan(chord, first, growth, s0, g, d_max)
    per = 2.03 * chord + 2 * math.pi * ds
    return float(np.sum(per / (s0 + g * ds)))


def naca_omesh(n_nodes_target: int = 200_000, chord: float = 200.0, radius_c: float = 20.0,
               first: float = 0.5, growth: float = 1.1, surface_ratio: float = 1.4,
               structured_layers: int = 4, jitter: float = 0.2, seed: int = 3) -> Mesh:
    """Seeded NACA0012 O-mesh of straight-sided P2 triangles.

    The airfoil (leading edge at the origin, chord along +x) sits in a roughly
    circular domain of radius ``radius_c`` chords around mid-chord.  Points lie
    on offset curves of the surface: the first offset at ``first``, offsets
    growing by ``growth`` until they match the tangential spacing
    s(d) = s0 + g d, with s0 = surface_ratio * first and g chosen so that the
    P2 node count is close to ``n_nodes_target``.  The innermost
    ``structured_layers`` offsets are left unjittered (near-wall orthogonal
    layers); further ones are jittered.  Delaunay triangulation, then the
    triangles inside the airfoil are dropped.  Every consecutive pair of
    surface points is checked to be a mesh edge.
    """
    rng = np.random.default_rng(seed)
    s0 = surface_ratio * first
    d_max = radius_c * chord - 0.5 * chord
    v_target = n_nodes_target / 4.0
    lo_g, hi_g = 1e-4, 2.0
    for _ in range(60):
        mid_g = math.sqrt(lo_g * hi_g)
        if _estimate_vertices(chord, first, growth, s0, mid_g, d_max) > v_target:
            lo_g = mid_g
        else:
            hi_g = mid_g
    g = math.sqrt(lo_g * hi_g)
    ds = _layer_plan(chord, first, growth, s0, g, d_max)
    poly = _airfoil_polygon(chord, s0)
    ns = poly.shape[0]
    layers = [poly]
    for j, d in enumerate(ds[1:], start=1):
        ht = s0 + g * d
        cur = _offset_curve(poly, d, dphi=min(0.04, 0.25 * ht / max(d, 1e-9)))
        phase = 0.0 if j <= structured_layers else rng.uniform(0.0, 1.0)
        pts = _resample_closed(cur, ht, phase)
        if structured_layers < j < len(ds) - 1:
            step = ds[j] - ds[j - 1]
            amp = jitter * min(ht, step)
            pts = pts + rng.uniform(-amp, amp, pts.shape)
        layers.append(pts)
    Xv = np.concatenate(layers, axis=0)
    n_outer = layers[-1].shape[0]
    V = Xv.shape[0]
    tri = Delaunay(Xv).simplices.astype(np.int64)
    # drop triangles inside the airfoil: only those with all vertices on the surface can be
    surf = np.all(tri < ns, axis=1)
    cen = Xv[tri].mean(axis=1)
    inside = np.zeros(tri.shape[0], dtype=bool)
    idx = np.nonzero(surf)[0]
    if idx.size:
        c = cen[idx]
        a = poly
        b = np.roll(poly, -1, axis=0)
        crs = ((b[None, :, 0] - a[None, :, 0]) * (c[:, None, 1] - a[None, :, 1])
               - (b[None, :, 1] - a[None, :, 1]) * (c[:, None, 0] - a[None, :, 0]))
        inside[idx] = np.all(crs > 0, axis=1)
    tri = tri[~inside]
    # surface edges must all be present
    edges = set()
    for k in range(3):
        a_ = tri[:, (k + 1) % 3]
        b_ = tri[:, (k + 2) % 3]
        m = (a_ < ns) & (b_ < ns)
        for u, v in zip(a_[m], b_[m]):
            edges.add((min(u, v), max(u, v)))
    for i in range(ns):
        u, v = i, (i + 1) % ns
        if (min(u, v), max(u, v)) not in edges:
            raise ValueError(f"surface edge {u}-{v} is not a Delaunay edge; refine the surface")
    outer0 = V - n_outer
    surf_next = {(i, (i + 1) % ns) for i in range(ns)}
    surf_next |= {(b, a) for (a, b) in surf_next}

    def tag(a, b):
        if (a, b) in surf_next:
            return WALL
        if a >= outer0 and b >= outer0:
            return FARFIELD
        raise ValueError(f"unexpected boundary edge {a}-{b}")

    m = _attach_p2(Xv, tri, np.zeros(2), tag)
    if m.wall_edges.shape[0] != ns:
        raise ValueError("wall edge count differs from surface point count")
    m.meta.update(kind="naca_omesh", chord=chord, radius_c=radius_c, first=first, growth=growth,
                  s0=s0, g=g, n_layers=len(ds), n_surface=ns, seed=seed)
    return m


def structured_square(nx: int, ny: int, Lx: float = 1.0, Ly: float = 1.0,
                      jitter: float = 0.0, seed: int = 0, tag=FARFIELD) -> Mesh:
    """Non-periodic P2 mesh of [0,Lx] x [0,Ly] (small test meshes): grid
    vertices, interior ones jittered by +-jitter spacings, Delaunay.  Every
    boundary edge gets ``tag``."""
    rng = np.random.default_rng(seed)
    xs = np.linspace(0.0, Lx, nx + 1)
    ys = np.linspace(0.0, Ly, ny + 1)
    P = np.stack(np.meshgrid(xs, ys, indexing="xy"), axis=-1).reshape(-1, 2)
    inner = (P[:, 0] > 0) & (P[:, 0] < Lx) & (P[:, 1] > 0) & (P[:, 1] < Ly)
    if jitter > 0:
        J = rng.uniform(-jitter, jitter, P.shape) * np.array([Lx / nx, Ly / ny])
        P[inner] += J[inner]
    else:
        P[inner] += 1e-9 * rng.uniform(-1, 1, (int(inner.sum()), 2))
    tri = Delaunay(P).simplices
    m = _attach_p2(P, tri, np.zeros(2), lambda a, b: tag)
    m.meta.update(kind="square", nx=nx, ny=ny, Lx=Lx, Ly=Ly)
    return m
