"""Pins of the oracle's layer algebra and per-label area.

Layer algebra follows set semantics on operand predicates (§3.4.2 names
logic operations between layers; §4.2 makes database-layer values unsigned
keys).  It is checked exhaustively over all 256 x 256 u8 value pairs against
Python set operations, and by identities.  Per-label areas are checked by
partition (bins sum to the covered area) and inclusion-exclusion.
"""

import itertools

import numpy as np
import pytest

import synth

AND, OR, XOR, REMAP = 0, 1, 2, 3


def _pred_set(vals, sel):
    return {t for t, v in enumerate(vals) if (v != 0 if sel == 0 else v == sel)}


@pytest.mark.parametrize("sel_a,sel_b", [(0, 0), (7, 0), (0, 200), (255, 1)])
def test_logic_ops_exhaustive_u8(orc, sel_a, sel_b):
    a = np.repeat(np.arange(256, dtype=np.uint8), 256)
    b = np.tile(np.arange(256, dtype=np.uint8), 256)
    Sa, Sb = _pred_set(a.tolist(), sel_a), _pred_set(b.tolist(), sel_b)
    for op, want in ((AND, Sa & Sb), (OR, Sa | Sb), (XOR, Sa ^ Sb)):
        dst = np.full(a.size, 99, np.uint8)
        orc.layer_op(op, dst, a, b, sel_a, sel_b, 42)
        got = set(np.nonzero(dst == 42)[0].tolist())
        assert got == want
        assert set(np.unique(dst).tolist()) <= {0, 42}


def test_logic_ops_mixed_dtypes_and_alias(orc):
    rng = np.random.default_rng(3)
    a = rng.integers(0, 4, 5000).astype(np.uint16) * 16000
    b = rng.integers(0, 3, 5000).astype(np.uint8)
    Sa, Sb = _pred_set(a.tolist(), 0), _pred_set(b.tolist(), 2)
    dst = b.copy()                          # dst aliases b in the call below
    orc.layer_op(OR, dst, a, dst, 0, 2, 250)
    assert set(np.nonzero(dst == 250)[0].tolist()) == Sa | Sb
    wide = np.zeros(5000, np.uint16)
    orc.layer_op(XOR, wide, a, b, 16000, 0, 60000)
    assert set(np.nonzero(wide == 60000)[0].tolist()) == _pred_set(a.tolist(), 16000) ^ _pred_set(b.tolist(), 0)


def test_logic_identities(orc):
    rng = np.random.default_rng(4)
    a = rng.integers(0, 6, 10000).astype(np.uint8)
    out = np.empty_like(a)
    orc.layer_op(XOR, out, a, a, 0, 0, 1)
    assert not out.any()
    orc.layer_op(AND, out, a, a, 0, 0, 1)
    assert np.array_equal(out == 1, a != 0)
    orc.layer_op(OR, out, a, a, 3, 3, 1)
    assert np.array_equal(out == 1, a == 3)


def test_remap_identity_and_composition(orc):
    rng = np.random.default_rng(5)
    for dt, n in ((np.uint8, 256), (np.uint16, 65536)):
        a = rng.integers(0, n, 20000).astype(dt)
        ident = np.arange(n, dtype=np.uint16)
        out = np.empty_like(a)
        orc.layer_op(REMAP, out, a, None, lut=ident)
        assert np.array_equal(out, a)
        f = np.concatenate([[0], 1 + rng.permutation(n - 1)]).astype(np.uint16)
        g = np.concatenate([[0], 1 + rng.permutation(n - 1)]).astype(np.uint16)
        o1, o2 = np.empty_like(a), np.empty_like(a)
        orc.layer_op(REMAP, o1, a, None, lut=f)
        orc.layer_op(REMAP, o2, o1, None, lut=g)
        gf = g[f]
        o3 = np.empty_like(a)
        orc.layer_op(REMAP, o3, a, None, lut=gf)
        assert np.array_equal(o2, o3)
        assert ((a == 0) == (o3 == 0)).all()
    with pytest.raises(ValueError):
        orc.layer_op(REMAP, out, a, None, lut=np.ones(65536, np.uint16))


@pytest.fixture(scope="module")
def vessel_geom(orc):
    return orc.geometry_image(synth.vessel(), 256, 256)


def test_area_partition_and_inclusion_exclusion(orc, vessel_geom):
    g = vessel_geom
    rng = np.random.default_rng(6)
    pts = synth.surface_points(rng, synth.vessel(), 12)
    A = np.zeros(g.tri_id.size, np.uint8)
    B = np.zeros(g.tri_id.size, np.uint8)
    for k, c in enumerate(pts):
        orc.brush(g.pos32, A if k % 2 else B, c, 0.4, 1 + k % 5)
    total = g.w[g.tri_id >= 0].sum()
    for L in (A, B):
        assert abs(orc.area(g, L).sum() / total - 1) < 1e-13
    U, I, X = (np.empty_like(A) for _ in range(3))
    orc.layer_op(OR, U, A, B, 0, 0, 1)
    orc.layer_op(AND, I, A, B, 0, 0, 1)
    orc.layer_op(XOR, X, A, B, 0, 0, 1)
    aA = orc.area(g, A)[1:].sum()
    aB = orc.area(g, B)[1:].sum()
    aU, aI, aX = (orc.area(g, L)[1] for L in (U, I, X))
    assert abs(aU - (aA + aB - aI)) < 1e-12 * total
    assert abs(aX - (aU - aI)) < 1e-12 * total
    # a single-label layer holds the whole covered area
    full = np.full(g.tri_id.size, 77, np.uint8)
    assert abs(orc.area(g, full)[77] / total - 1) < 1e-14


def test_area_u16_bins(orc, vessel_geom):
    g = vessel_geom
    L = (np.arange(g.tri_id.size) % 65536).astype(np.uint16)
    a = orc.area(g, L)
    assert a.shape == (65536,)
    for l in (0, 1, 300, 65535):
        assert abs(a[l] - g.w[L == l].sum()) < 1e-12
