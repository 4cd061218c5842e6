"""Numeric layers in the CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module; the product library never does.

The paper keeps two kinds of information layer (§4.2): database layers,
whose data texture holds unsigned primary keys, and numeric layers, which
hold integer or real properties (curvature, age, ...).  A layer is a data
texture of 8-, 16- or 32-bit integers or 16- or 32-bit floats plus a mask
texture of booleans telling which texels hold valid data.  Readings used
here (the paper gives the textures, not the operations on numeric layers):

  - dtypes: unsigned 8 and 16 bit, signed 32 bit, IEEE binary16 and
    binary32 (codes U8=1, U16=2, I32=3, F16=4, F32=5);
  - the mask is one bit per texel, texel t = j W + i in bit t mod 32 of
    32-bit word t div 32;
  - an edit selects texels exactly as the label edits do (brush, lasso,
    screen-space tool of §4.3.1) and then either SETs them (data = the value
    converted to the layer's dtype, mask bit = 1) or ERASEs them (mask bit =
    0, data untouched); the value is converted once: integers must be exact
    and in range, floats round to nearest, ties to even, and must stay
    finite;
  - texture padding (§4.3.2) of a numeric layer SETs or ERASEs the
    outline texels the label padding would label;
  - a range selection turns quantitative data into a label: texels whose
    mask bit is set and whose value v (exact in fp64) satisfies
    lo <= v <= hi take the label in a label layer; others keep theirs;
  - zonal statistics over the texels that a triangle covers and whose mask
    bit is set, grouped by the value of a label layer (one group when there
    is none): count, surface area, area-weighted sum of values, minimum and
    maximum.  Table 1 gives the surface area one texel stands for; the
    weighted sum over the area is the area-weighted mean;
  - operations between two numeric layers of one dtype, texel by texel
    (operating with quantitative information, §4.2): a result validity r
    (AND / OR / XOR of the operands' mask bits; both valid for MIN, MAX and
    ADD); where r holds, the data become the value (mask operations: a's
    value if a is valid, else b's; MIN: a if a <= b else b; MAX: a if
    a >= b else b; ADD: the sum rounded once to the dtype -- integers
    exactly, binary32 by its own addition, binary16 from the exact sum --
    with results beyond the dtype's finite range taking its extreme finite
    value); where r does not hold, the data stay and the bit is cleared.

Pins (tests/test_oracle_numeric.py): binary16 bit patterns fixed by the
IEEE 754 format (normal, subnormal, ties, overflow) and numpy's independent
conversion on random values; a hand-packed mask; SET then ERASE; the
discrete moments of x and x^2 over a facing plane in closed form (mean,
minimum, maximum, per-quadrant means); the area of a range selection.
"""

from __future__ import annotations

import math

import numpy as np

from . import brush as _brush, lasso as _lasso, pad as _pad, tool as _tool

U8, U16, I32, F16, F32 = 1, 2, 3, 4, 5
SET, ERASE = 0, 1
NUM_AND, NUM_OR, NUM_XOR, NUM_MIN, NUM_MAX, NUM_ADD = 0, 1, 2, 3, 4, 5

NP_DTYPE = {U8: np.uint8, U16: np.uint16, I32: np.int32, F16: np.float16, F32: np.float32}
INT_RANGE = {U8: (0, 255), U16: (0, 65535), I32: (-2 ** 31, 2 ** 31 - 1)}


def f16_bits(x: float) -> int:
    """IEEE binary16 bit pattern of the double x, rounded to nearest with
    ties to even (§4.2 lists 16-bit floats).  Raises OverflowError when the
    result is not finite.  From the format: 1 sign bit, 5 exponent bits
    (bias 15), 10 fraction bits; subnormals below 2^-14 with spacing 2^-24."""
    if not math.isfinite(x):
        raise OverflowError("not finite")
    sign = 0x8000 if math.copysign(1.0, x) < 0 else 0
    a = abs(x)
    if a == 0.0:
        return sign
    e = max(math.frexp(a)[1] - 1, -14)          # a in [2^e, 2^(e+1)) for normals
    ulp = 2.0 ** (e - 10)
    q = round(a / ulp)                          # exact scaling; round() is half-even
    if q == 2048:                               # rounded up to the next binade
        e, q = e + 1, 1024
    if e > 15:
        raise OverflowError("beyond binary16")
    if q < 1024:                                # subnormal (e == -14)
        return sign | q
    return sign | ((e + 15) << 10) | (q - 1024)


def encode(value: float, dtype: int):
    """The stored value of `value` in `dtype` as a numpy scalar; ValueError
    if it does not fit (integers: not integral or out of range; floats: not
    finite after rounding)."""
    value = float(value)
    if math.isnan(value):
        raise ValueError("NaN")
    if dtype in INT_RANGE:
        lo, hi = INT_RANGE[dtype]
        if value != math.floor(value) or not lo <= value <= hi:
            raise ValueError(f"{value} does not fit dtype {dtype}")
        return NP_DTYPE[dtype](int(value))
    if dtype == F16:
        try:
            return np.array(f16_bits(value), np.uint16).view(np.float16)[()]
        except OverflowError as e:
            raise ValueError(str(e)) from None
    if dtype == F32:
        with np.errstate(over="ignore"):
            v = np.float32(value)              # round to nearest even
        if not np.isfinite(v):
            raise ValueError("beyond binary32")
        return v
    raise ValueError(f"dtype {dtype}")


def pack_mask(valid: np.ndarray) -> np.ndarray:
    """Bit t of the word array (bit t mod 32 of word t div 32) = valid[t]."""
    v = np.asarray(valid, bool).reshape(-1)
    nw = (v.size + 31) // 32
    bits = np.zeros(nw * 32, np.uint64)
    bits[:v.size] = v
    weights = np.uint64(1) << np.arange(32, dtype=np.uint64)
    return (bits.reshape(nw, 32) * weights).sum(axis=1).astype(np.uint32)


def unpack_mask(words: np.ndarray, n: int) -> np.ndarray:
    w = np.asarray(words, np.uint32).astype(np.uint64)
    bits = (w[:, None] >> np.arange(32, dtype=np.uint64)) & np.uint64(1)
    return bits.reshape(-1)[:n].astype(bool)


class NumericLayer:
    """Data texture (numpy array of the dtype) and mask texture (bool per
    texel) of one numeric layer, both flat over the W x H atlas."""

    def __init__(self, n: int, dtype: int):
        self.dtype = dtype
        self.data = np.zeros(n, NP_DTYPE[dtype])
        self.valid = np.zeros(n, bool)

    @property
    def words(self) -> np.ndarray:
        return pack_mask(self.valid)


def apply(layer: NumericLayer, sel: np.ndarray, mode: int, value: float = 0.0) -> int:
    """Write one edit's selection (bool per texel) into the layer."""
    sel = np.asarray(sel, bool)
    if mode == SET:
        layer.data[sel] = encode(value, layer.dtype)
        layer.valid[sel] = True
    elif mode == ERASE:
        layer.valid[sel] = False
    else:
        raise ValueError("mode")
    return int(sel.sum())


def brush(pos32, layer: NumericLayer, centre, radius, mode: int, value: float = 0.0) -> int:
    sel = np.zeros(layer.data.size, np.uint8)
    _brush(pos32, sel, centre, radius, 1)
    return apply(layer, sel == 1, mode, value)


def lasso(pos32, layer: NumericLayer, M, poly, depth, bias, mode: int, value: float = 0.0) -> int:
    sel = np.zeros(layer.data.size, np.uint8)
    _lasso(pos32, sel, M, poly, depth, bias, 1)
    return apply(layer, sel == 1, mode, value)


def tool(pos32, layer: NumericLayer, M, tool_params, shape, depth, bias, mode: int, value: float = 0.0) -> int:
    sel = np.zeros(layer.data.size, np.uint8)
    _tool(pos32, sel, M, tool_params, shape, depth, bias, 1)
    return apply(layer, sel == 1, mode, value)


def pad(outline_mask, edited, W: int, H: int, k: int, layer: NumericLayer, mode: int, value: float = 0.0) -> int:
    """Texture padding of a numeric layer after one edit (§4.3.2): the
    outline texels the label padding would label are SET or ERASEd."""
    sel = np.zeros(layer.data.size, np.uint8)
    _pad(outline_mask, edited, W, H, k, sel, 1)
    return apply(layer, sel == 1, mode, value)


def select(layer: NumericLayer, lo: float, hi: float, dst: np.ndarray, label: int) -> int:
    """Range selection into a label layer, in place."""
    v = layer.data.astype(np.float64)
    hit = layer.valid & (v >= lo) & (v <= hi)
    dst[hit] = label
    return int(hit.sum())


STATS_DTYPE = np.dtype([("count", np.uint64), ("area", np.float64), ("wsum", np.float64),
                        ("vmin", np.float64), ("vmax", np.float64), ("abs_wsum", np.float64),
                        ("abs_vsum", np.float64)])


def stats(tri_id: np.ndarray, w: np.ndarray, layer: NumericLayer, region=None) -> np.ndarray:
    """Zonal statistics: one record per value of `region` (a u8 or u16 label
    layer; one record when it is None).  Over covered texels (tri_id >= 0)
    with the mask bit set: count, area = sum of the fp64 texel areas w,
    wsum = sum of w v (each product rounded once, the sum correctly rounded
    by math.fsum), vmin, vmax (+inf / -inf when empty).  abs_wsum = sum
    |w v| and abs_vsum = sum |v| bound the rounding of other summation
    orders and of quantised areas."""
    nb = 1 if region is None else (256 if region.dtype == np.uint8 else 65536)
    lab = np.zeros(layer.data.size, np.int64) if region is None else np.asarray(region).astype(np.int64)
    keep = (np.asarray(tri_id) >= 0) & layer.valid
    v = layer.data.astype(np.float64)
    out = np.zeros(nb, STATS_DTYPE)
    out["vmin"] = np.inf
    out["vmax"] = -np.inf
    w = np.asarray(w, np.float64)
    idx = np.flatnonzero(keep)
    idx = idx[np.argsort(lab[idx], kind="stable")]          # texels grouped by label
    for grp in np.split(idx, np.flatnonzero(np.diff(lab[idx])) + 1):
        if grp.size == 0:
            continue
        vb, wb = v[grp], w[grp]
        out[lab[grp[0]]] = (grp.size, math.fsum(wb), math.fsum(wb * vb), vb.min(), vb.max(),
                            math.fsum(np.abs(wb * vb)), math.fsum(np.abs(vb)))
    return out


FLOAT_MAX = {F16: 65504.0, F32: float(np.finfo(np.float32).max)}


def _add(xa: np.ndarray, xb: np.ndarray, dtype: int) -> np.ndarray:
    """Saturating sum in the dtype: integers exact, then clipped to the
    range; binary32 by its own (correctly rounded) addition; binary16 from
    the exact sum (in fp64) rounded once; float results beyond the largest
    finite value take it, with their sign."""
    if dtype in INT_RANGE:
        lo, hi = INT_RANGE[dtype]
        return np.clip(xa.astype(np.int64) + xb.astype(np.int64), lo, hi).astype(NP_DTYPE[dtype])
    with np.errstate(over="ignore", invalid="ignore"):
        if dtype == F32:
            s = xa.astype(np.float32) + xb.astype(np.float32)
        else:
            s = (xa.astype(np.float64) + xb.astype(np.float64)).astype(np.float16)
    m = FLOAT_MAX[dtype]
    return np.where(np.isinf(s), np.copysign(m, s), s).astype(NP_DTYPE[dtype])


def combine(op: int, dst: NumericLayer, a: NumericLayer, b: NumericLayer) -> int:
    """dst = a op b texel by texel (dst may be a or b); returns the number
    of valid result texels."""
    if not (a.dtype == b.dtype == dst.dtype):
        raise ValueError("dtypes differ")
    va, vb = a.valid.copy(), b.valid.copy()
    xa, xb = a.data.copy(), b.data.copy()
    if op == NUM_AND:
        r = va & vb
    elif op == NUM_OR:
        r = va | vb
    elif op == NUM_XOR:
        r = va ^ vb
    elif op in (NUM_MIN, NUM_MAX, NUM_ADD):
        r = va & vb
    else:
        raise ValueError("op")
    if op in (NUM_AND, NUM_OR, NUM_XOR):
        val = np.where(va, xa, xb)
    elif op == NUM_MIN:
        val = np.where(xa <= xb, xa, xb)
    elif op == NUM_MAX:
        val = np.where(xa >= xb, xa, xb)
    else:
        val = _add(xa, xb, a.dtype)
    dst.data[r] = val[r]
    dst.valid[:] = r
    return int(r.sum())
