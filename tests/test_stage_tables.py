"""LDS staging tables (host side, no GPU): every ELL slot of every row must
read, through its LDS slot, exactly the column the pattern holds.

Both forms are checked by brute force against the mesh connectivity on
periodic grids in the caller's row order (two uneven instances, ragged
tiles): a row's slots, mapped through the stage a tile (form 2) or a
64-row wavefront (form 3) builds (its own rows, then its list), give the
row and its element neighbours.  In the Z-curve order the two forms must
give the same column sets row by row, and form 3 must address only its own
wavefront's rows and its own 192 halo slots.
"""
import numpy as np
import pytest

from paper_1608_01906_amd import felbm
from paper_1608_01906_amd.inputs import grid_mesh_2d, grid_mesh_3d

TILE = 256


def _neighbour_sets(mesh):
    n = mesh["xyz"].shape[0]
    nb = [set([k]) for k in range(n)]
    for el in mesh["conn"]:
        for a in el:
            nb[a].update(int(b) for b in el)
    return nb


def _context(meshes, node_order, **opts):
    ctx = felbm.Context(9, max_instances=len(meshes), node_order=node_order, **opts)
    for i, m in enumerate(meshes):
        ctx.upload_mesh(i, m)
    return ctx


def _columns(tab, form, rows):
    """Global column read by every (slot, row) through the form's stage."""
    lcol, ptr, col = tab["lcol"].astype(np.int64), tab["list_ptr"], tab["list_col"]
    W, R = lcol.shape
    r = np.arange(R)
    tile = r // TILE
    out = np.empty((W, R), np.int64)
    for k in range(W):
        s = lcol[k]
        own = s < TILE
        out[k, own] = tile[own] * TILE + s[own]
        h = ~own
        if form == 2:
            entry = ptr[tile[h]] + (s[h] - TILE)
            assert np.all(s[h] - TILE < np.diff(ptr)[tile[h]])
        else:
            w = (s[h] - TILE) // 192
            assert np.all(w == (r[h] % TILE) // 64), "a wavefront reads another wavefront's halo slots"
            wv = tile[h] * 4 + w
            entry = ptr[wv] + (s[h] - TILE) % 192
            assert np.all((s[h] - TILE) % 192 < np.diff(ptr)[wv])
        out[k, h] = col[entry]
    if form == 3:
        own = lcol < TILE
        assert np.all((lcol[own] // 64) == ((r[None, :] % TILE) // 64 * np.ones_like(lcol))[own]), \
            "form 3 reads a row of another wavefront from its own slot"
    return out


def _check_lists(tab, unit):
    ptr, col = tab["list_ptr"], tab["list_col"]
    for u in range(len(ptr) - 1):
        c = col[ptr[u]:ptr[u + 1]]
        assert np.all(np.diff(c) > 0)
        assert not np.any((c >= u * unit) & (c < (u + 1) * unit))
        if unit == 64:
            assert len(c) <= 192


def test_stage_tables_caller_order():
    meshes = [grid_mesh_2d(37, 29, jitter=0.2, seed=5), grid_mesh_2d(20, 20, jitter=0.2, seed=6)]
    ctx = _context(meshes, 0)
    info = ctx.layout_info()
    R = info["rows"]
    starts = np.cumsum([0] + [-(-m["xyz"].shape[0] // TILE) * TILE for m in meshes])
    for form, unit in ((2, TILE), (3, 64)):
        tab = ctx.stage_tables(form)
        _check_lists(tab, unit)
        got = _columns(tab, form, R)
        for i, m in enumerate(meshes):
            nb = _neighbour_sets(m)
            b = starts[i]
            for k in range(m["xyz"].shape[0]):
                assert set((got[:, b + k] - b).tolist()) == nb[k], (form, i, k)
            # padding rows read themselves only
            pad = np.arange(b + m["xyz"].shape[0], starts[i + 1])
            assert np.all(got[:, pad] == pad[None, :])
    assert starts[-1] == R


def test_stage_tables_zcurve_forms_agree():
    meshes = [grid_mesh_2d(45, 33, jitter=0.2, seed=7), grid_mesh_2d(64, 64, jitter=0.2, seed=8)]
    ctx = _context(meshes, 1)
    t2, t3 = ctx.stage_tables(2), ctx.stage_tables(3)
    _check_lists(t2, TILE)
    _check_lists(t3, 64)
    g2, g3 = _columns(t2, 2, None), _columns(t3, 3, None)
    np.testing.assert_array_equal(np.sort(g2, axis=0), np.sort(g3, axis=0))
    # an interior wavefront of the curve order is an 8 x 8 block of nodes:
    # halo of 4 sides of 8 and the 2 corners the P1 split's diagonal reaches
    assert np.median(np.diff(t3["list_ptr"])) == 34


def test_stage_tables_availability():
    ctx = _context([grid_mesh_2d(16, 16)], 0, lds_staging=1)
    ctx.stage_tables(2)
    with pytest.raises(felbm.FelError):  # not built for a schedule that never uses it
        ctx.stage_tables(3)
    c3 = felbm.Context(19)
    c3.upload_mesh(0, grid_mesh_3d(6, 6, 6))
    c3.stage_tables(2)
    with pytest.raises(felbm.FelError):  # ELL width 15: no per-wavefront form
        c3.stage_tables(3)
    for bad in (0, 1, 4):
        with pytest.raises(felbm.FelError):
            ctx.stage_tables(bad)


def test_scattered_numbering_has_no_wavefront_form():
    """A grid whose nodes are numbered at random, kept in the caller's order:
    a 64-row wavefront then references about 6 x 64 other rows, more than
    its 192 halo slots, so the per-wavefront tables are not built (form 3 is
    refused); the per-tile tables still map every slot to its column."""
    m = grid_mesh_2d(40, 40, jitter=0.0)
    rng = np.random.default_rng(5)
    perm = rng.permutation(m["xyz"].shape[0])
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    shuffled = dict(m, xyz=m["xyz"][perm], conn=inv[m["conn"]].astype(m["conn"].dtype))
    for key in ("wall", "wall_normal"):
        if key in m:
            shuffled[key] = m[key][perm]
    ctx = _context([shuffled], 0)
    with pytest.raises(felbm.FelError):
        ctx.stage_tables(3)
    t2 = ctx.stage_tables(2)
    got = _columns(t2, 2, None)
    nb = _neighbour_sets(shuffled)
    for k in range(shuffled["xyz"].shape[0]):
        assert set(got[:, k].tolist()) == nb[k]
