"""Correctly rounded FP32 fused multiply-add on numpy arrays.

Test infrastructure: used by the oracle's FP32 association decisions, which are
defined with fused multiply-adds (one rounding per a*b + c, IEEE 754 fusedMultiplyAdd
in binary32, round to nearest, ties to even).

Method.  The product of two binary32 values is exact in binary64 (at most 48
significant bits).  s = fl64(p + c) rounds once; its exact error e = (p + c) - s
follows from Knuth's TwoSum.  Rounding s to binary32 gives the correct result
unless s lies exactly halfway between two adjacent binary32 values while the exact
sum does not (double rounding): binary32 midpoints are binary64 numbers and
rounding is monotonic, so p + c and s are then on the same side of every other
boundary.  In that case the result is the neighbour on the side of e.
"""
import numpy as np

f32 = np.float32
f64 = np.float64


def fma32(a, b, c):
    """round_to_binary32(a * b + c) computed exactly, elementwise (a, b, c are
    binary32 scalars or arrays; returns binary32)."""
    a64 = np.asarray(a, dtype=f32).astype(f64)
    b64 = np.asarray(b, dtype=f32).astype(f64)
    c64 = np.asarray(c, dtype=f32).astype(f64)
    with np.errstate(all="ignore"):
        p = a64 * b64                      # exact
        s = p + c64
        bv = s - p                         # TwoSum: e = (p + c) - s exactly
        av = s - bv
        e = (p - av) + (c64 - bv)
        r = s.astype(f32)
        r64 = r.astype(f64)
        up = np.nextafter(r, f32(np.inf))
        dn = np.nextafter(r, f32(-np.inf))
        lo = np.where(r64 > s, dn, r)      # binary32 neighbours around s
        hi = np.where(r64 > s, r, up)
        tie = (s != r64) & (2.0 * s == lo.astype(f64) + hi.astype(f64)) & np.isfinite(s)
        out = np.where(tie & (e > 0), hi, np.where(tie & (e < 0), lo, r))
    return out.astype(f32)
