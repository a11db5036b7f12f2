"""C-ABI checks that need no GPU: exported symbols, argument validation, and the
library's host-side domain builder against the oracle's geometry (step a1)."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import grid

sa = pytest.importorskip("paper_0907_4863_amd")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "saamg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(saamg_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = sa.capi.lib()
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n


def test_default_options_follow_table1():
    o = sa.default_options()
    assert o.max_coarse == 1000 and o.cheb_degree == 2 and o.precision == sa.FP64
    assert abs(o.omega_scale - 4.0 / 3.0) < 1e-15


@pytest.mark.parametrize("shape,n,nz", [
    (W.Shape.cylinder(1.0, 2.0), 33, 33),
    (W.Shape.ellipse(1.0, 0.6, 4.0), 64, 96),
    (W.Shape.boxbore(0.8, 4.0, 0.5), 47, 93),
    (W.Shape.cylinder(0.5, 1.0), 65, 65),
    (W.Shape.cylinder(1.0, 6.0), 83, 9),  # lattice points exactly on the wall
])
def test_domain_builder_matches_oracle(shape, n, nz):
    d = sa.domain_for(shape, n, n, nz)
    o = grid.from_shape(shape, n, n, nz)
    assert np.array_equal(d.mask.astype(bool), o.mask)
    we = grid.wall_entries(o)
    assert np.array_equal(d.wall_node, we["node"])
    assert np.array_equal(d.wall_dir, we["dir"])
    assert np.max(np.abs(d.wall_s - we["s"]), initial=0.0) <= 1e-14


@pytest.mark.parametrize("shape,n,nz", [
    (W.Shape.cylinder(1.0, 2.0), 33, 21),
    (W.Shape.ellipse(1.0, 0.6, 4.0), 40, 30),
    (W.Shape.boxbore(0.8, 4.0, 0.5), 31, 45),
    (W.Shape(W.BOXBORE, 1.0, 0.7, 2.0, 0.1, 2.0), 9, 11),  # cavity through the ends
])
def test_domain_builder_open_ends_matches_oracle(shape, n, nz):
    d = sa.domain_for(shape, n, n, nz, open_ends=True)
    o = grid.from_shape(shape, n, n, nz, robin=True)
    assert d.mask.shape == (nz + 2, n, n) and d.robin_d == 0.5 * shape.length == o.robin_d
    assert np.array_equal(d.mask.astype(bool), o.mask)
    we = grid.wall_entries(o)
    assert np.array_equal(d.wall_node, we["node"])
    assert np.array_equal(d.wall_dir, we["dir"])
    assert np.max(np.abs(d.wall_s - we["s"]), initial=0.0) <= 1e-14


def test_domain_builder_open_ends_paper_dof_count():
    d = sa.domain_from_shape(sa.capi.SHAPE_CYLINDER, 1.0, 1.0, 2.0, 128, 128, 256, open_ends=True)
    assert d.n_unknowns == 3236864


def test_domain_builder_paper_dof_count():
    d = sa.domain_from_shape(sa.capi.SHAPE_CYLINDER, 1.0, 1.0, 2.0, 33, 33, 33)
    assert d.n_unknowns == 24583


def _dom(mask, node=(), dr=(), s=()):
    return sa.capi.HostDomain(mask, (0.1, 0.1, 0.1), np.array(node, np.int64),
                              np.array(dr, np.uint8), np.array(s, np.float64))


def test_setup_rejects_invalid_domains_before_touching_the_gpu():
    m = np.zeros((5, 5, 5), np.uint8)
    with pytest.raises(sa.SaamgError, match="no unknowns"):
        sa.setup(_dom(m), sa.VARIANT_LIN)
    m2 = m.copy()
    m2[0, 2, 2] = 1
    with pytest.raises(sa.SaamgError, match="face"):
        sa.setup(_dom(m2), sa.VARIANT_LIN)
    m3 = m.copy()
    m3[2, 2, 2] = 1
    with pytest.raises(sa.SaamgError, match="fraction"):
        sa.setup(_dom(m3, [62], [0], [0.0]), sa.VARIANT_LIN)
    with pytest.raises(sa.SaamgError, match="neighbour"):
        m4 = m.copy()
        m4[2, 2, 2] = m4[2, 2, 1] = 1
        sa.setup(_dom(m4, [62], [0], [0.5]), sa.VARIANT_LIN)
    with pytest.raises(sa.SaamgError, match="duplicate"):
        sa.setup(_dom(m3, [62, 62], [0, 0], [0.5, 0.5]), sa.VARIANT_QUAD)
    with pytest.raises(sa.SaamgError, match="variant"):
        sa.setup(_dom(m3), 7)
    with pytest.raises(sa.SaamgError, match="cheb_degree"):
        sa.setup(_dom(m3), sa.VARIANT_LIN, sa.default_options(cheb_degree=0))
    assert "cheb_degree" in sa.capi.last_error()
    bad = _dom(m3)
    bad.robin_d = -1.0
    with pytest.raises(sa.SaamgError, match="robin_d"):
        sa.setup(bad, sa.VARIANT_LIN)
    lonely = m.copy()
    lonely[1, 2, 2] = 1  # end-plane unknown with nothing inside
    op = _dom(lonely)
    op.robin_d = 1.0
    with pytest.raises(sa.SaamgError, match="open-end"):
        sa.setup(op, sa.VARIANT_LIN)


def test_footprint_grows_with_box_and_precision():
    h64, s64 = sa.footprint_bytes(128, 128, 256, sa.VARIANT_QUAD, sa.FP64)
    hm, sm = sa.footprint_bytes(128, 128, 256, sa.VARIANT_QUAD, sa.MIXED)
    h2, s2 = sa.footprint_bytes(256, 256, 768, sa.VARIANT_QUAD, sa.MIXED)
    assert s64 > sm > 0 and h2 > hm and s2 > sm
    assert s64 >= 48 * 128 * 128 * 256


def test_refresh_rejects_a_null_hierarchy_before_touching_the_gpu():
    m = np.zeros((5, 5, 5), np.uint8)
    m[2, 2, 2] = 1
    H = sa.capi.Hierarchy(0, (5, 5, 5))
    with pytest.raises(sa.SaamgError, match="hierarchy is NULL"):
        sa.refresh(H, _dom(m))


def test_wall_entries_in_any_order_are_checked_for_duplicates():
    m = np.zeros((5, 5, 5), np.uint8)
    m[2, 2, 2] = 1
    with pytest.raises(sa.SaamgError, match="duplicate"):
        sa.setup(_dom(m, [62, 62, 62], [1, 0, 1], [0.5, 0.5, 0.5]), sa.VARIANT_QUAD)
    # unsorted and distinct: the host checks pass (without a GPU the call then fails later)
    try:
        H = sa.setup(_dom(m, [62, 62], [1, 0], [0.5, 0.5]), sa.VARIANT_QUAD)
        sa.destroy(H)
    except sa.SaamgError as e:
        assert "duplicate" not in str(e) and "wall" not in str(e)
