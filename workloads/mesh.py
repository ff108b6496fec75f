"""Extruded-mesh descriptions (input data only).

A mesh is a horizontal tessellation (1D intervals for a vertical x-z slice,
quadrilaterals for a 3D domain) that is extruded into ``nz`` layers, in the
spirit of the paper's extruded meshes (Sec. 3.1.2).  The description carries:

* ``eh_nodes``  [n_eh, (p+1)^(dim-1)] int32: global horizontal node id of every
  element-local GLL node.  Local order: ``i`` (along xi) fastest, then ``j``
  (along eta).  Periodic identification is folded into these ids.
* ``eh_corner`` [n_eh, 2^(dim-1), dim-1] float64: *unwrapped* physical corner
  coordinates.  Quad corners are ordered (-1,-1), (+1,-1), (+1,+1), (-1,+1) in
  reference coordinates; interval corners are (-1), (+1).
* ``eh_arc``    [n_eh, 4, 3] float64 or None: per quad edge, (cx, cy, R) of a
  circle the edge follows (R = 0: straight).  Edges are e0: c0->c1 (eta=-1),
  e1: c1->c2 (xi=+1), e2: c3->c2 (eta=+1), e3: c0->c3 (xi=-1); an arc edge is
  parametrised linearly in angle along the shorter arc between its corners.
* ``eh_face_tag`` [n_eh, 2(dim-1)] int32: per side face, 0 interior/periodic,
  1 impermeable wall, 2 body.  Sides are ordered like the edges above for
  quads, and (xi=-1, xi=+1) for intervals.

GLL node positions are *not* part of the description: every consumer maps
the reference GLL points through the corner/arc (Gordon-Hall) description
itself.  The numbering is pure combinatorics (vertex / edge / interior).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

TAG_INTERIOR = 0
TAG_WALL = 1
TAG_BODY = 2


@dataclass
class HexMesh:
    dim: int
    p: int
    nz: int
    n_s: int
    eh_nodes: np.ndarray
    eh_corner: np.ndarray
    eh_face_tag: np.ndarray
    eh_arc: Optional[np.ndarray] = None
    layer_s: Optional[np.ndarray] = None
    # periodic lengths (Lx, Ly) used only for consistency checks; 0 = not periodic
    period: tuple = (0.0, 0.0)
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n_eh(self) -> int:
        return int(self.eh_nodes.shape[0])

    @property
    def nh(self) -> int:
        return (self.p + 1) ** (self.dim - 1)

    @property
    def n_lev(self) -> int:
        """Number of vertical node levels, p*nz + 1."""
        return self.p * self.nz + 1

    @property
    def n_v(self) -> int:
        return self.n_s * self.n_lev

    @property
    def n_e(self) -> int:
        return self.n_eh * self.nz

    def layer_fractions(self) -> np.ndarray:
        if self.layer_s is not None:
            return np.asarray(self.layer_s, dtype=np.float64)
        return np.arange(self.nz + 1, dtype=np.float64) / self.nz


def structured_slice(nx: int, x0: float, x1: float, periodic: bool, p: int, nz: int, name: str = "") -> HexMesh:
    """Vertical x-z slice: ``nx`` intervals on [x0, x1], extruded in ``nz`` layers."""
    if periodic and nx < 3:
        raise ValueError("periodic meshes need at least 3 elements across the period")
    n1 = p + 1
    n_i = p * nx + (0 if periodic else 1)
    e = np.arange(nx)[:, None]
    i = np.arange(n1)[None, :]
    nodes = (e * p + i) % n_i
    dx = (x1 - x0) / nx
    corner = np.zeros((nx, 2, 1))
    corner[:, 0, 0] = x0 + dx * np.arange(nx)
    corner[:, 1, 0] = x0 + dx * (np.arange(nx) + 1)
    tags = np.zeros((nx, 2), dtype=np.int32)
    if not periodic:
        tags[0, 0] = TAG_WALL
        tags[-1, 1] = TAG_WALL
    return HexMesh(dim=2, p=p, nz=nz, n_s=n_i, eh_nodes=nodes.astype(np.int32), eh_corner=corner,
                   eh_face_tag=tags, period=((x1 - x0) if periodic else 0.0, 0.0), name=name,
                   extra=dict(nx=nx, x0=x0, x1=x1))


def structured_box(nx: int, ny: int, x0: float, x1: float, y0: float, y1: float,
                   periodic_x: bool, periodic_y: bool, p: int, nz: int, name: str = "") -> HexMesh:
    """Rectangle [x0,x1]x[y0,y1] split into nx*ny axis-aligned quads (x fastest)."""
    if (periodic_x and nx < 3) or (periodic_y and ny < 3):
        raise ValueError("periodic meshes need at least 3 elements across the period")
    n1 = p + 1
    n_ix = p * nx + (0 if periodic_x else 1)
    n_iy = p * ny + (0 if periodic_y else 1)
    ex = np.tile(np.arange(nx), ny)
    ey = np.repeat(np.arange(ny), nx)
    i = np.tile(np.arange(n1), n1)
    j = np.repeat(np.arange(n1), n1)
    gi = (ex[:, None] * p + i[None, :]) % n_ix
    gj = (ey[:, None] * p + j[None, :]) % n_iy
    nodes = gj * n_ix + gi
    dx = (x1 - x0) / nx
    dy = (y1 - y0) / ny
    xa = x0 + dx * ex
    xb = x0 + dx * (ex + 1)
    ya = y0 + dy * ey
    yb = y0 + dy * (ey + 1)
    corner = np.stack([np.stack([xa, ya], -1), np.stack([xb, ya], -1),
                       np.stack([xb, yb], -1), np.stack([xa, yb], -1)], axis=1)
    tags = np.zeros((nx * ny, 4), dtype=np.int32)
    if not periodic_y:
        tags[ey == 0, 0] = TAG_WALL
        tags[ey == ny - 1, 2] = TAG_WALL
    if not periodic_x:
        tags[ex == nx - 1, 1] = TAG_WALL
        tags[ex == 0, 3] = TAG_WALL
    return HexMesh(dim=3, p=p, nz=nz, n_s=n_ix * n_iy, eh_nodes=nodes.astype(np.int32), eh_corner=corner,
                   eh_face_tag=tags,
                   period=((x1 - x0) if periodic_x else 0.0, (y1 - y0) if periodic_y else 0.0), name=name,
                   extra=dict(nx=nx, ny=ny, x0=x0, x1=x1, y0=y0, y1=y1, n_ix=n_ix, n_iy=n_iy))


def quad_mesh_from_vertices(vert_xy: np.ndarray, quads: np.ndarray, p: int, nz: int,
                            arcs: Optional[np.ndarray] = None, face_tag: Optional[np.ndarray] = None,
                            name: str = "") -> HexMesh:
    """High-order horizontal numbering of an unstructured (non-periodic) quad mesh.

    ``quads`` [n_eh, 4] are counter-clockwise vertex ids.  Global horizontal
    node ids are: vertices (by vertex id), then (p-1) nodes per edge for edges
    in order of first appearance (oriented from the lower to the higher vertex
    id), then (p-1)^2 interior nodes per element (row-major in (j, i)).
    """
    quads = np.asarray(quads, dtype=np.int64)
    n_vert = int(vert_xy.shape[0])
    n_eh = int(quads.shape[0])
    n1 = p + 1
    nodes = np.full((n_eh, n1 * n1), -1, dtype=np.int64)
    edge_base = {}
    next_id = n_vert
    # local corner positions (i, j)
    cpos = [(0, 0), (p, 0), (p, p), (0, p)]
    # edges: (start corner, end corner, function t -> (i, j)) along increasing local index
    edefs = [(0, 1, lambda t: (t, 0)), (1, 2, lambda t: (p, t)), (3, 2, lambda t: (t, p)), (0, 3, lambda t: (0, t))]
    for e in range(n_eh):
        vs = quads[e]
        for c in range(4):
            i, j = cpos[c]
            nodes[e, j * n1 + i] = vs[c]
        for (ca, cb, pos) in edefs:
            a, b = int(vs[ca]), int(vs[cb])
            if a == b:
                raise ValueError("degenerate edge")
            key = (min(a, b), max(a, b))
            if key not in edge_base:
                edge_base[key] = next_id
                next_id += p - 1
            base = edge_base[key]
            for t in range(1, p):
                i, j = pos(t)
                nodes[e, j * n1 + i] = base + (t - 1 if a < b else p - 1 - t)
    for e in range(n_eh):
        for j in range(1, p):
            for i in range(1, p):
                nodes[e, j * n1 + i] = next_id
                next_id += 1
    assert (nodes >= 0).all()
    corner = vert_xy[quads]  # [n_eh, 4, 2]
    tags = np.zeros((n_eh, 4), dtype=np.int32) if face_tag is None else np.asarray(face_tag, dtype=np.int32)
    return HexMesh(dim=3, p=p, nz=nz, n_s=int(next_id), eh_nodes=nodes.astype(np.int32),
                   eh_corner=np.ascontiguousarray(corner, dtype=np.float64), eh_face_tag=tags,
                   eh_arc=None if arcs is None else np.ascontiguousarray(arcs, dtype=np.float64), name=name,
                   extra=dict(vert_xy=vert_xy, quads=quads))


def cylinder_tank_mesh(p: int = 4, nz: int = 4, seed: int = 0, n_theta: int = 48, n_rad: int = 24,
                       radius: float = 0.25, tank=(10.0, 5.0), spacing: float = 1.0 / 6.0,
                       hole_half: float = 1.0, jitter: float = 0.1, name: str = "cylinder_tank") -> HexMesh:
    """Bottom-mounted vertical cylinder in a rectangular tank.

    An O-grid of ``n_theta`` x ``n_rad`` quads around the cylinder (circle
    edges exact, straight radial lines to the square hole boundary, blended
    linearly in the radial index) is joined to a Cartesian block of spacing
    ``spacing`` with the square hole cut out.  Interior block vertices are
    jittered uniformly in [-jitter, jitter] * spacing per coordinate.
    """
    lx, ly = tank
    nbx = int(round(lx / spacing))
    nby = int(round(ly / spacing))
    cx, cy = lx / 2.0, ly / 2.0
    hx0 = int(round((cx - hole_half) / spacing))
    hx1 = int(round((cx + hole_half) / spacing))
    hy0 = int(round((cy - hole_half) / spacing))
    hy1 = int(round((cy + hole_half) / spacing))
    side = hx1 - hx0
    assert side == hy1 - hy0 and 4 * side == n_theta, "square hole sides must carry n_theta/4 cells"
    rng = np.random.default_rng(seed)

    # block vertices
    vid = -np.ones((nbx + 1, nby + 1), dtype=np.int64)
    verts = []
    for J in range(nby + 1):
        for I in range(nbx + 1):
            inside_hole = hx0 < I < hx1 and hy0 < J < hy1
            if inside_hole:
                continue
            vid[I, J] = len(verts)
            verts.append((I * spacing, J * spacing))
    verts = np.array(verts, dtype=np.float64)
    # jitter interior block vertices (not on the tank boundary, not on the hole boundary)
    jit = rng.uniform(-jitter, jitter, size=verts.shape) * spacing
    movable = np.zeros(len(verts), dtype=bool)
    for J in range(nby + 1):
        for I in range(nbx + 1):
            v = vid[I, J]
            if v < 0:
                continue
            on_tank = I in (0, nbx) or J in (0, nby)
            on_hole = (hx0 <= I <= hx1 and hy0 <= J <= hy1)
            movable[v] = not (on_tank or on_hole)
    verts[movable] += jit[movable]

    quads, tags, arcs = [], [], []
    for J in range(nby):
        for I in range(nbx):
            if hx0 <= I < hx1 and hy0 <= J < hy1:
                continue
            quads.append((vid[I, J], vid[I + 1, J], vid[I + 1, J + 1], vid[I, J + 1]))
            t = [TAG_INTERIOR] * 4
            if J == 0:
                t[0] = TAG_WALL
            if I == nbx - 1:
                t[1] = TAG_WALL
            if J == nby - 1:
                t[2] = TAG_WALL
            if I == 0:
                t[3] = TAG_WALL
            tags.append(t)
            arcs.append(np.zeros((4, 3)))

    # hole boundary, counter-clockwise starting at the lower-right corner
    ring = []
    for k in range(side):
        ring.append((hx1, hy0 + k))
    for k in range(side):
        ring.append((hx1 - k, hy1))
    for k in range(side):
        ring.append((hx0, hy1 - k))
    for k in range(side):
        ring.append((hx0 + k, hy0))
    outer_ids = np.array([vid[I, J] for (I, J) in ring])
    outer_xy = verts[outer_ids]
    theta = np.arctan2(outer_xy[:, 1] - cy, outer_xy[:, 0] - cx)
    circ = np.stack([cx + radius * np.cos(theta), cy + radius * np.sin(theta)], -1)
    # O-grid vertices: rings r = 0 (circle) .. n_rad (square); ring n_rad reuses block ids
    ogrid_id = np.zeros((n_rad + 1, n_theta), dtype=np.int64)
    ogrid_id[n_rad] = outer_ids
    new_verts = []
    base = len(verts)
    for r in range(n_rad):
        s = r / n_rad
        for t in range(n_theta):
            ogrid_id[r, t] = base + len(new_verts)
            new_verts.append((1.0 - s) * circ[t] + s * outer_xy[t])
    verts = np.concatenate([verts, np.array(new_verts)], axis=0)
    for r in range(n_rad):
        for t in range(n_theta):
            t1 = (t + 1) % n_theta
            quads.append((ogrid_id[r, t], ogrid_id[r + 1, t], ogrid_id[r + 1, t1], ogrid_id[r, t1]))
            tg = [TAG_INTERIOR] * 4
            a = np.zeros((4, 3))
            if r == 0:
                tg[3] = TAG_BODY
                a[3] = (cx, cy, radius)
            tags.append(tg)
            arcs.append(a)
    quads = np.array(quads, dtype=np.int64)
    m = quad_mesh_from_vertices(verts, quads, p, nz, arcs=np.array(arcs), face_tag=np.array(tags), name=name)
    m.extra.update(dict(tank=tank, center=(cx, cy), radius=radius, n_block=int(len(quads) - n_theta * n_rad)))
    return m


def renumber_blocked(m: HexMesh, shared_first: bool = False) -> HexMesh:
    """The same mesh with its horizontal nodes renumbered column by column.

    Every node goes to the lowest-numbered horizontal element (column) that has it; each
    column's nodes get consecutive ids, the ones it shares with other columns first, then its
    interior ones, both in local order.  A volume vector (layer-major) then holds each
    column's own nodes at a node level as one contiguous run, and the shared ones of a column
    as a shorter run at its start.  shared_first: all shared nodes (column by column) before
    all interior nodes, so the shared nodes of a node level form one contiguous range.
    """
    import dataclasses
    nodes = m.eh_nodes.astype(np.int64)
    n_eh, nh = nodes.shape
    g = nodes.ravel()
    col = np.repeat(np.arange(n_eh), nh)
    loc = np.tile(np.arange(nh), n_eh)
    owner = np.full(m.n_s, n_eh, dtype=np.int64)
    np.minimum.at(owner, g, col)
    count = np.bincount(g, minlength=m.n_s)
    mine = col == owner[g]
    og, oloc = g[mine], loc[mine]
    key_col = owner[og]
    key_int = (count[og] == 1).astype(np.int64)
    order = np.lexsort((oloc, key_col, key_int)) if shared_first else np.lexsort((oloc, key_int, key_col))
    new = np.empty(m.n_s, dtype=np.int64)
    new[og[order]] = np.arange(og.size)
    extra = dict(m.extra)
    extra["numbering"] = "blocked-shared-first" if shared_first else "blocked"
    return dataclasses.replace(m, eh_nodes=new[nodes].astype(np.int32), extra=extra)
