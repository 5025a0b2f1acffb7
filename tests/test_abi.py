"""C ABI of libfelbm.so without a GPU: every declared symbol is exported,
and the host-side validation (options, mesh checks, layout sizing) returns
the documented status codes.  No device call is made here."""
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1608_01906_amd import felbm
from paper_1608_01906_amd.inputs import grid_mesh_2d, grid_mesh_3d

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "felbm.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"FEL_API[^;]*?\b(fel_[a-z_]+)\s*\(", text, re.S)))


def test_all_declared_symbols_exported():
    declared = _declared()
    assert len(declared) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", felbm.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (fel_[a-z_]+)", out))
    assert set(declared) <= exported, set(declared) - exported
    assert sorted(felbm.ABI_SYMBOLS) == declared
    assert felbm.load_library().fel_version().startswith(b"felbm")


def test_bad_options_rejected():
    for kw in [dict(precision="fp64", max_instances=0)]:
        with pytest.raises(felbm.FelError):
            felbm.Context(9, **kw)
    with pytest.raises(felbm.FelError):
        felbm.Context(7)
    for nb in (3, 8, -1):
        with pytest.raises(felbm.FelError):
            felbm.Context(9, solver_batch=nb)
    for sg in (4, -1):
        with pytest.raises(felbm.FelError):
            felbm.Context(9, lds_staging=sg)
    for fr in (3, -1):
        with pytest.raises(felbm.FelError):
            felbm.Context(9, fused_reductions=fr)


def test_tuning_before_bind():
    """A fixed solver schedule shows on the solver kernels at once; 0 (timed
    at the first step) reads 0 until then; the streaming kernel (batch 1)
    takes the staging option too (its staged form is per tile, so 3 reads
    2), which binding settles to direct where it has no staged form; other
    kernels read (1, 1)."""
    solver = ("cg_init", "cg_a", "cg_b", "cheb")
    for nb in (0, 1, 2, 4):
        for sg in (0, 1, 2, 3):
            t = felbm.Context(19, solver_batch=nb, lds_staging=sg).tuning()
            assert all(t[k] == (nb, sg) for k in solver)
            assert t["stream"] == (1, min(sg, 2))
            assert all(v == (1, 1) for k, v in t.items() if k not in solver and k not in ("stream", "fused"))
            assert t["fused"] == 0


def test_halo_lists():
    """Per-tile halos of the LDS stage, brute force on a small periodic grid:
    a 16 x 16 row-major block of a 32 x 32 grid in caller order has as halo
    the 32-node rows above and below plus the wrap-around columns."""
    ctx = felbm.Context(9, node_order=0)
    ctx.upload_mesh(0, grid_mesh_2d(32, 32, jitter=0.0))
    info = ctx.layout_info()
    # tile = grid rows 8k .. 8k + 7 (256 nodes); neighbours of the P1 split
    # with diagonal (0,0)-(1,1) reach one grid row up and down: 2 x 32
    assert info["halo_max"] == 64 and info["halo_mean"] == 64.0
    z = felbm.Context(9, node_order=1)
    z.upload_mesh(0, grid_mesh_2d(32, 32, jitter=0.0))
    zi = z.layout_info()
    # Z-order tiles are 16 x 16 blocks: 4 sides of 16 plus 2 corners
    assert zi["halo_max"] == 66 and zi["halo_mean"] == 66.0


def test_inverted_element_rejected():
    m = grid_mesh_2d(4, 4)
    m["conn"] = m["conn"][:, [0, 2, 1]].copy()
    m["shift"] = m["shift"][:, [0, 2, 1]].copy()
    ctx = felbm.Context(9)
    with pytest.raises(felbm.FelError) as ei:
        ctx.upload_mesh(0, m)
    assert ei.value.status == felbm.FEL_EINVAL


def test_index_out_of_range_rejected():
    m = grid_mesh_2d(4, 4)
    m["conn"] = m["conn"].copy()
    m["conn"][3, 1] = 16
    ctx = felbm.Context(9)
    with pytest.raises(felbm.FelError) as ei:
        ctx.upload_mesh(0, m)
    assert ei.value.status == felbm.FEL_EINVAL


def test_dimension_mismatch_and_order():
    ctx = felbm.Context(9, max_instances=2)
    with pytest.raises(felbm.FelError):
        ctx.upload_mesh(0, grid_mesh_3d(3, 3, 3))
    with pytest.raises(felbm.FelError):
        ctx.upload_mesh(2, grid_mesh_2d(4, 4))
    # step before bind
    ctx.upload_mesh(0, grid_mesh_2d(4, 4))
    with pytest.raises(felbm.FelError) as ei:
        ctx.step(1)
    assert ei.value.status == felbm.FEL_ESTATE


def test_layout_padding_and_workspace():
    ctx = felbm.Context(9, max_instances=3)
    sizes = [(5, 5), (20, 13), (16, 16)]
    for i, (a, b) in enumerate(sizes):
        ctx.upload_mesh(i, grid_mesh_2d(a, b, seed=i))
    info = ctx.layout_info()
    assert info["rows"] == 256 * (1 + 2 + 1)   # every instance starts on a 256-row tile
    assert info["ell_width"] == 7 and info["pops"] == 18 and info["cg_iters"] == 30
    assert ctx.workspace_size() > 0
    c3 = felbm.Context(19, precision="fp32")
    c3.upload_mesh(0, grid_mesh_3d(4, 4, 4))
    info = c3.layout_info()
    assert info["ell_width"] == 15 and info["cg_iters"] == 17


def test_valence_above_widest_layout_rejected():
    """A 3-D Delaunay mesh with a node of valence 26 exceeds the widest ELL
    layout (24 slots): the layout is refused with FEL_EINVAL."""
    from paper_1608_01906_amd.inputs.mesh import delaunay_mesh
    ctx = felbm.Context(19)
    ctx.upload_mesh(0, delaunay_mesh((10, 10, 10), seed=1618))
    with pytest.raises(felbm.FelError) as ei:
        ctx.layout_info()
    assert ei.value.status == felbm.FEL_EINVAL
    ok = felbm.Context(19)
    ok.upload_mesh(0, delaunay_mesh((10, 10, 10), seed=1614))
    assert ok.layout_info()["ell_width"] == 24
