"""FP8 operand encoding of the precision form's all-pairs screen (oracle).

Test infrastructure only: the library never imports this module.

OCP 8-bit floating point, E4M3 variant: 1 sign bit, 4 exponent bits with
bias 7, 3 mantissa bits; exponent field 0 holds the subnormals m * 2^-9; the
code with all exponent and mantissa bits set is NaN; there are no
infinities, so the largest finite magnitude is 1.75 * 2^8 = 448.

The screen scales each row a_i by s_i = max_l |a_il| / 448 (FP32 division;
s_i = 1 for a zero row), rounds every a_il / s_i (FP32 division) to the
nearest e4m3 value (ties to the even code, magnitudes beyond 448 saturate to
448), and keeps N_i = s_i^2 |q_i|^2 (the squared norm of the decoded row in
FP64, times the exact FP64 square of s_i, rounded once).

This module writes the encoding out as its definition: the table of the 127
non-negative finite values, a nearest-value search with even-code ties.
"""
import numpy as np

E4M3_MAX = 448.0


def decode(code):
    """Value of e4m3 byte(s) (NaN for 0x7F / 0xFF)."""
    c = np.asarray(code, dtype=np.int64)
    sign = np.where(c & 0x80, -1.0, 1.0)
    e = (c >> 3) & 0xF
    m = c & 0x7
    val = np.where(e == 0, m * 2.0 ** -9, (1.0 + m / 8.0) * np.exp2(e - 7.0))
    val = np.where((c & 0x7F) == 0x7F, np.nan, val)
    return sign * val


_CODES = np.arange(0x7F)          # non-negative finite codes, increasing value
_VALUES = decode(_CODES)


def encode(x):
    """Nearest e4m3 code of each FP32/FP64 value (ties to the even code,
    saturating at +-448).  The sign bit is kept when a negative value rounds
    to zero (0x80, negative zero); +0 and -0 themselves encode to 0x00."""
    x = np.asarray(x, dtype=np.float64)
    a = np.minimum(np.abs(x), E4M3_MAX)
    hi = np.clip(np.searchsorted(_VALUES, a, side="left"), 0, len(_VALUES) - 1)
    lo = np.maximum(hi - 1, 0)
    dlo = np.abs(a - _VALUES[lo])
    dhi = np.abs(_VALUES[hi] - a)
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (_CODES[hi] % 2 == 0))
    code = np.where(pick_hi, _CODES[hi], _CODES[lo])
    return (code | np.where(x < 0, 0x80, 0)).astype(np.uint8)


def quantize_rows(A):
    """(Q, s, N) of the FP32 rows of A: Q[i] = e4m3(fl32(a_i / s_i)),
    s_i = fl32(max |a_i| / 448) (1 for a zero row), N_i = fl64(sum_l
    decode(Q[i, l])^2 * s_i^2)."""
    A = np.asarray(A, dtype=np.float32)
    mx = np.abs(A).max(axis=1)
    s = np.where(mx > 0, mx / np.float32(E4M3_MAX), np.float32(1.0)).astype(np.float32)
    ratio = (A / s[:, None]).astype(np.float32)
    Q = encode(ratio)
    v = decode(Q)
    N = (v * v).sum(axis=1) * (s.astype(np.float64) ** 2)
    return Q, s, N
