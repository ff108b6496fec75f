"""Mesh and numbering pins: the paper's printed DoF counts, Euler's relation, geometric consistency."""

import json
import os

import numpy as np
import pytest

from oracle import geometry as geo
from workloads import configs, mesh as wm

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "dof_tables.json")))


@pytest.mark.parametrize("row", GOLD["periodic_boxes"], ids=lambda r: r["cite"])
def test_periodic_tables(row):
    nx, ny = row["n"]
    m = wm.structured_box(nx, ny, 0.0, float(nx), 0.0, float(ny), True, True, p=row["p"], nz=row["nz"])
    assert m.n_s == row["dof_surface"]
    assert m.n_v == row["dof_volume"]
    if m.n_eh <= 40000:
        assert np.unique(m.eh_nodes).size == m.n_s


@pytest.mark.parametrize("row", GOLD["walled_boxes"], ids=lambda r: r["cite"])
def test_walled_tables(row):
    nx, ny = row["n"]
    m = wm.structured_box(nx, ny, 0.0, 38.0, 0.0, 1.0, False, False, p=row["p"], nz=row["nz"])
    assert m.n_s == row["dof_surface"]
    assert m.n_v == row["dof_volume"]


@pytest.mark.parametrize("row", GOLD["column_factor"], ids=lambda r: r["cite"])
def test_column_factor(row):
    lev = row["p"] * row["nz"] + 1
    assert row["dof_volume"] % lev == 0
    if "dof_surface" in row:
        assert row["dof_surface"] * lev == row["dof_volume"]


def test_config_counts():
    assert configs.c1().mesh.n_v == 288
    assert configs.c2().mesh.n_v == 840000
    m4 = configs.c4().mesh
    assert (m4.n_s, m4.n_v) == (26001, 546021)
    m5 = configs.c5().mesh
    assert (m5.n_s, m5.n_v, m5.n_e) == (1180416, 43675392, 196608)
    assert configs.p1().mesh.n_v == 1114112


def test_cylinder_mesh_topology():
    m = configs.c3().mesh
    quads = m.extra["quads"]
    assert m.n_eh == 48 * 24 + 60 * 30 - 144 == 2808
    edges = set()
    for q in quads:
        for a, b in ((0, 1), (1, 2), (2, 3), (3, 0)):
            edges.add((min(q[a], q[b]), max(q[a], q[b])))
    V = len(np.unique(quads))
    E = len(edges)
    F = len(quads)
    assert V - E + F == 0          # planar domain with one hole
    p = m.p
    assert m.n_s == V + (p - 1) * E + (p - 1) ** 2 * F
    assert m.n_v == m.n_s * (p * m.nz + 1)
    # counter-clockwise quads everywhere (positive horizontal Jacobian)
    xh = geo.horizontal_coords(m)
    geo.check_numbering(m, xh)


@pytest.mark.parametrize("name", ["C1", "C2", "C4", "P1"])
def test_numbering_consistency(name):
    m = configs.ALL[name]().mesh
    geo.check_numbering(m)


def test_numbering_inconsistency_detected():
    m = wm.structured_box(4, 3, 0.0, 2.0, 0.0, 1.5, True, False, p=3, nz=1)
    bad = m.eh_nodes.copy()
    bad[0, 1], bad[0, 3] = bad[0, 3], bad[0, 1]      # node 3 is shared with the next element
    m.eh_nodes = bad
    with pytest.raises(ValueError):
        geo.check_numbering(m)


def test_layer_major_surface_slice():
    m = configs.c1().mesh
    dofs = geo.dof_map(m)
    top = dofs.reshape(m.n_e, m.p + 1, m.p + 1)[m.nz - 1::m.nz, m.p, :]
    # the top node level of the top layer is the contiguous slice [p nz n_s, (p nz + 1) n_s)
    assert top.min() == m.p * m.nz * m.n_s and top.max() == m.n_v - 1


@pytest.mark.parametrize("periodic", [(True, False), (False, False), (True, True)])
def test_renumber_blocked(periodic):
    """Blocked numbering: a consistent bijection; each column's own nodes are one run, shared first."""
    m = wm.structured_box(5, 4, 0.0, 2.0, 0.0, 1.5, periodic[0], periodic[1], p=3, nz=2)
    b = wm.renumber_blocked(m)
    geo.check_numbering(b)
    # the same physical node at every (column, local node)
    perm = np.full(m.n_s, -1)
    perm[m.eh_nodes.ravel()] = b.eh_nodes.ravel()
    assert np.all(np.sort(perm) == np.arange(m.n_s))
    assert np.all(perm[m.eh_nodes] == b.eh_nodes)
    counts = np.bincount(b.eh_nodes.ravel(), minlength=b.n_s)
    nxt = 0
    for e in range(b.n_eh):
        ids = b.eh_nodes[e]
        owned = [g for g in ids if not np.any(b.eh_nodes[:e] == g)]
        assert sorted(owned) == list(range(nxt, nxt + len(owned)))
        shared = [g for g in owned if counts[g] > 1]
        assert sorted(shared) == list(range(nxt, nxt + len(shared)))
        nxt += len(owned)
    assert nxt == b.n_s


@pytest.mark.parametrize("periodic", [(False, False), (True, False), (True, True)])
def test_renumber_shared_first(periodic):
    """Shared-first blocked numbering: a consistent bijection with every shared node before every
    interior node, each group column by column (owner order) as one run per column."""
    m = wm.structured_box(5, 4, 0.0, 2.0, 0.0, 1.5, periodic[0], periodic[1], p=3, nz=2)
    b = wm.renumber_blocked(m, shared_first=True)
    geo.check_numbering(b)
    perm = np.full(m.n_s, -1)
    perm[m.eh_nodes.ravel()] = b.eh_nodes.ravel()
    assert np.all(np.sort(perm) == np.arange(m.n_s))
    counts = np.bincount(b.eh_nodes.ravel(), minlength=b.n_s)
    n_shared = int((counts > 1).sum())
    assert np.all(counts[:n_shared] > 1) and np.all(counts[n_shared:] == 1)
    nxt_s, nxt_i = 0, n_shared
    for e in range(b.n_eh):
        ids = b.eh_nodes[e]
        owned = [g for g in ids if not np.any(b.eh_nodes[:e] == g)]
        sh = sorted(g for g in owned if counts[g] > 1)
        it = sorted(g for g in owned if counts[g] == 1)
        assert sh == list(range(nxt_s, nxt_s + len(sh))) and it == list(range(nxt_i, nxt_i + len(it)))
        nxt_s += len(sh)
        nxt_i += len(it)
    assert nxt_s == n_shared and nxt_i == b.n_s


def test_apply_invariant_under_renumbering():
    """The oracle's apply commutes with a renumbering of the horizontal nodes."""
    from oracle import operator as op
    wl = configs.small_box(nx=4, ny=3, nz=2, p=3, periodic=(True, False))
    m = wl.mesh
    b = wm.renumber_blocked(m)
    perm = np.full(m.n_s, -1)
    perm[m.eh_nodes.ravel()] = b.eh_nodes.ravel()
    levels = m.p * m.nz + 1
    vperm = (np.arange(levels)[:, None] * m.n_s + perm[None, :]).ravel()   # old volume index -> new
    x, y = geo.node_xy(m)
    h, eta = wl.depth(x, y), wl.eta0(x, y)
    G, _, _ = geo.factors(m, eta, h)
    xb_pos = geo.node_xy(b)
    Gb, _, _ = geo.factors(b, eta[np.argsort(perm)], h[np.argsort(perm)])
    rng = np.random.default_rng(5)
    u = rng.standard_normal(m.n_v)
    ub = np.empty_like(u)
    ub[vperm] = u
    ya = op.apply(m, G, u)
    yb = op.apply(b, Gb, ub)
    assert np.abs(yb[vperm] - ya).max() < 1e-13 * np.abs(ya).max()
    assert np.abs(xb_pos[0][perm] - x).max() < 1e-14


@pytest.mark.parametrize("periodic", [False, True])
def test_node_coords_tensor_grid(periodic):
    """Horizontal node coordinates of an axis-aligned box: the tensor product of the GLL points
    mapped into each interval (x_e + (1 + xi_i) dx / 2), every node listed once (the first image
    on a periodic axis)."""
    from oracle.gll import gll
    nx, ny, p = 4, 3, 3
    x0, x1, y0, y1 = -1.0, 3.0, 0.5, 2.0
    m = wm.structured_box(nx, ny, x0, x1, y0, y1, periodic, periodic, p=p, nz=1)
    xi, _, _ = gll(p)
    dx, dy = (x1 - x0) / nx, (y1 - y0) / ny

    def axis(n, a, d, per):
        pts = sorted({round(a + (e + (1 + s) / 2) * d, 12) for e in range(n) for s in xi})
        if per:
            pts = [q for q in pts if q < a + n * d - 1e-9]   # the period's end is its start
        return np.array(pts)

    gx, gy = axis(nx, x0, dx, periodic), axis(ny, y0, dy, periodic)
    c = geo.node_coords(m)
    assert c.shape == (len(gx) * len(gy), 2) and not np.isnan(c).any()
    want = np.array([(a, b) for a in gx for b in gy])
    key = lambda z: np.lexsort((np.round(z[:, 1], 9), np.round(z[:, 0], 9)))
    assert np.abs(c[key(c)] - want[key(want)]).max() < 1e-12


def test_sigma_levels_closed_form():
    """sigma at level v = l p + k: s_l + (1 + xi_k)(s_{l+1} - s_l) / 2, from 0 at the bottom to 1
    at the surface, increasing, with the layer boundaries shared."""
    from oracle.gll import gll
    m = wm.structured_box(3, 3, 0.0, 1.0, 0.0, 1.0, False, False, p=4, nz=3)
    m.layer_s = np.array([0.0, 0.2, 0.65, 1.0])
    xi, _, _ = gll(4)
    sig = geo.sigma_levels(m)
    want = np.array([m.layer_s[l] + (1 + xi[k]) * (m.layer_s[l + 1] - m.layer_s[l]) / 2
                     for l in range(3) for k in range(4)] + [1.0])
    assert sig.shape == (m.n_lev,)
    assert np.abs(sig - want).max() < 1e-15
    assert sig[0] == 0.0 and sig[-1] == 1.0 and np.all(np.diff(sig) > 0)
