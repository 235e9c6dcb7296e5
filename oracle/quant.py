"""Reduced-precision formats and the emulated reduced-precision preconditioner.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Section 3 (after eq. (PreconSolve)) stores V_r, V_c and S in 16-bit half
precision and computes the preconditioner solve in it; Section 4 simulates
that with a rounding function applied after each operation.  This module
provides the rounding functions and an emulation of the preconditioner chain
as a reduced-precision implementation runs it:

  * operands (V, the scaled residual, and each intermediate product) are
    rounded to the storage format;
  * each product is formed exactly (FP64 here), i.e. this emulates storage
    rounding, not low-precision accumulation (an implementation accumulates
    in FP32; the tests allow for that with an explicit accumulation bound).

Formats:
  * FP16: IEEE binary16, round to nearest even, with subnormals
    (numpy.float16), max 65504.
  * FP8 e4m3 ("e4m3fn"): 1 sign, 4 exponent (bias 7), 3 mantissa bits; no
    infinities; S.1111.111 is NaN, so the largest finite value is
    1.75 * 2^8 = 448; subnormals (m/8) * 2^-6; round to nearest even;
    values beyond 448 saturate to 448.  Written from that definition and
    pinned against an independent library cast over all 256 codes.

Precision reading (Section 3 stores S in FP16): S = 1/(s^2 + lambda^2)
overflows FP16 for lambda < 3.9e-3, so the FP16 chain folds lambda^2 into
S' = lambda^2 S in (0, 1] and scales r by a power of two so that the scaled
residual has 2-norm below 2^14; orthogonality of V then keeps every FP16
intermediate below 65504.  z = Z' / (scale * lambda^2).

The FP8 chain uses block scaling: each run of 32 consecutive entries along
the contracted dimension of an operand shares a power-of-two scale chosen so
that the run's largest magnitude maps to at most 448.
"""
from __future__ import annotations

import math

import numpy as np

FP16_MAX = 65504.0
E4M3_MAX = 448.0
FP16_SCALE_TARGET_LOG2 = 14
FP8_BLOCK = 32


def round_fp16(x):
    return np.asarray(x, dtype=np.float64).astype(np.float16).astype(np.float64)


def round_fp32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_e4m3(x):
    """Round to the nearest e4m3 value (ties to even), saturating at +-448."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    nan = np.isnan(x)
    a = np.abs(np.where(nan, 0.0, x))
    # quantum: 2^-9 in the subnormal range (|x| < 2^-6), else 2^(E-3)
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    e = np.clip(e, -6, 8)
    q = np.exp2(e - 3)
    m = np.rint(a / q) * q          # np.rint rounds half to even
    m = np.minimum(m, E4M3_MAX)
    out[:] = np.copysign(m, x)
    out[nan] = np.nan
    return out


def e4m3_decode(code: int) -> float:
    """Value of an 8-bit e4m3 code, from the format definition."""
    s = -1.0 if code & 0x80 else 1.0
    e = (code >> 3) & 0xF
    m = code & 0x7
    if e == 0xF and m == 0x7:
        return math.nan
    if e == 0:
        return s * (m / 8.0) * 2.0 ** -6
    return s * (1.0 + m / 8.0) * 2.0 ** (e - 7)


def pow2_scale_for_norm(norm: float, target_log2: int = FP16_SCALE_TARGET_LOG2) -> float:
    """Power of two s with s * norm < 2^target (and >= 2^(target-1))."""
    if not (norm > 0.0) or not math.isfinite(norm):
        return 1.0
    _, e = math.frexp(norm)          # norm = m 2^e, 0.5 <= m < 1
    return math.ldexp(1.0, target_log2 - e)


def block_exponents(x: np.ndarray, axis: int, block: int = FP8_BLOCK, vmax: float = E4M3_MAX):
    """Per-block power-of-two exponents along `axis` (blocks of `block`
    consecutive entries): the smallest e with max|x_block| * 2^-e <= vmax.
    Zero blocks get exponent -127.  Returns an integer array with the block
    index in place of `axis`."""
    x = np.moveaxis(np.asarray(x, dtype=np.float64), axis, -1)
    k = x.shape[-1]
    nb = (k + block - 1) // block
    pad = nb * block - k
    xp = np.pad(np.abs(x), [(0, 0)] * (x.ndim - 1) + [(0, pad)])
    amax = xp.reshape(x.shape[:-1] + (nb, block)).max(axis=-1)
    e = np.full(amax.shape, -127, dtype=np.int64)
    nz = amax > 0
    m, ee = np.frexp(amax[nz] / vmax)     # amax/vmax = m 2^ee, m in [0.5,1)
    ee = ee.astype(np.int64)
    ee[m == 0.5] -= 1                     # exact power of two fits one lower
    e[nz] = ee
    return np.moveaxis(e, -1, axis)


def quantize_e4m3_blocks(x: np.ndarray, axis: int, block: int = FP8_BLOCK):
    """(codes as float64 values, exponents): x ~ codes * 2^e per block."""
    e = block_exponents(x, axis, block)
    ef = np.repeat(e, block, axis=axis)
    sl = [slice(None)] * x.ndim
    sl[axis] = slice(0, x.shape[axis])
    ef = ef[tuple(sl)].astype(np.float64)
    q = round_e4m3(np.asarray(x, dtype=np.float64) * np.exp2(-ef))
    return q, e


def dequant(q: np.ndarray, e: np.ndarray, axis: int, block: int = FP8_BLOCK):
    ef = np.repeat(e, block, axis=axis).astype(np.float64)
    sl = [slice(None)] * q.ndim
    sl[axis] = slice(0, q.shape[axis])
    return q * np.exp2(ef[tuple(sl)])


# --------------------------------------------------------------------------
# emulated preconditioner chains, Z = V_c (S .* (V_c^T R V_r)) V_r^T
# --------------------------------------------------------------------------

def s_prime(sc, sr, lam):
    """S' = lambda^2 S = lambda^2 / (s_c^2 s_r^2 + lambda^2), in FP32 as an
    implementation computes it from FP32 squared singular values."""
    sc2 = round_fp32(np.asarray(sc) ** 2)
    sr2 = round_fp32(np.asarray(sr) ** 2)
    l2 = np.float32(lam * lam)
    den = (sc2[:, None].astype(np.float32) * sr2[None, :].astype(np.float32)) + l2
    return (l2 / den).astype(np.float64)


def precond_fp32(Vc, Vr, sc, sr, lam, r):
    """FP32-stored factors, exact products: the reference an FP32 chain is
    compared against (with an accumulation bound)."""
    vc, vr = round_fp32(Vc), round_fp32(Vr)
    t = vc.T @ round_fp32(r) @ vr
    t2 = s_prime(sc, sr, lam) * t
    return vc @ t2 @ vr.T / (lam * lam)


def precond_fp16(Vc, Vr, sc, sr, lam, r, rnorm=None):
    """FP16 chain with power-of-two residual scaling and S' folding; every
    intermediate that an implementation stores in FP16 is rounded to FP16."""
    r = np.asarray(r, dtype=np.float64)
    if rnorm is None:
        rnorm = float(np.linalg.norm(r))
    s = pow2_scale_for_norm(rnorm)
    vc, vr = round_fp16(Vc), round_fp16(Vr)
    rt = round_fp16(s * r)
    t1 = round_fp16(vc.T @ rt)
    t2 = round_fp16(s_prime(sc, sr, lam) * (t1 @ vr))
    t3 = round_fp16(vc @ t2)
    return (t3 @ vr.T) / (s * lam * lam)


def precond_fp8(Vc, Vr, sc, sr, lam, r):
    """FP8-e4m3 chain with 32-entry block scales along each contraction."""
    def left(x):     # contraction over columns (axis 1)
        q, e = quantize_e4m3_blocks(x, axis=1)
        return dequant(q, e, axis=1)

    def right(x):    # contraction over rows (axis 0)
        q, e = quantize_e4m3_blocks(x, axis=0)
        return dequant(q, e, axis=0)

    r = np.asarray(r, dtype=np.float64)
    t1 = left(Vc.T) @ right(r)
    t = left(t1) @ right(Vr)
    t2 = s_prime(sc, sr, lam) * t
    t3 = left(Vc) @ right(t2)
    return (left(t3) @ right(Vr.T)) / (lam * lam)


def gamma(k: int, u: float) -> float:
    """Higham's gamma_k = k u / (1 - k u)."""
    return k * u / (1.0 - k * u)


def fp32_chain_bound(Vc, Vr, sc, sr, lam, r):
    """First-order elementwise bound on |z_fp32_accumulated - z_exact_products|
    for the FP32 chain (standard dot-product error bound, gamma_n per GEMM,
    plus one FP32 rounding of each stored intermediate and of S')."""
    n = Vc.shape[0]
    u = 2.0 ** -24
    g = gamma(n, u) + u
    avc, avr = np.abs(round_fp32(Vc)), np.abs(round_fp32(Vr))
    ar = np.abs(round_fp32(r))
    sp = s_prime(sc, sr, lam)
    b1 = avc.T @ ar                 # |T1| bound
    e1 = g * b1                     # error of T1
    bt = b1 @ avr                   # |T| bound
    et = e1 @ avr + g * bt          # error of T
    e2 = sp * et + 2 * u * sp * bt  # error of T2 (S' rounding included)
    b2 = sp * bt
    e3 = avc @ e2 + g * (avc @ b2)
    b3 = avc @ b2
    ez = e3 @ avr.T + g * (b3 @ avr.T)
    return ez / (lam * lam)
