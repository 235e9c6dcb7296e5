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

Parity status: pinned (tests/test_oracle_quant.py).  The e4m3 codec against
an independent library table over all 256 codes and its cast; the block
quantiser against an entry-by-entry loop from the format definition, on a
ragged case where row and column blocking differ; both chains against the
FP64 preconditioner solve bit for bit on exact-product inputs (signed
permutation factors, S' in {1, 1/2}); the FP16 chain at every stored
operand against a 2 x 2 case worked by hand on rounding ties, and against
CPython's binary16 packing of each exact product; the FP8 chain at every
stored operand against the entry-by-entry quantiser.  The elementwise bounds
at the end of the module are checked against chains run with float32
products.
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


def precond_fp16(Vc, Vr, sc, sr, lam, r, rnorm=None, trace=None):
    """FP16 chain with power-of-two residual scaling and S' folding; every
    intermediate that an implementation stores in FP16 is rounded to FP16.
    `trace` (a dict, optional) receives the scale and every stored operand:
    scale, vc, vr, rt = fp16(scale r), t1 = fp16(Vc^T rt), t2 =
    fp16(S' .* (t1 Vr)), t3 = fp16(Vc t2)."""
    r = np.asarray(r, dtype=np.float64)
    if rnorm is None:
        rnorm = float(np.linalg.norm(r))
    s = pow2_scale_for_norm(rnorm)
    vc, vr = round_fp16(Vc), round_fp16(Vr)
    rt = round_fp16(s * r)
    t1 = round_fp16(vc.T @ rt)
    t2 = round_fp16(s_prime(sc, sr, lam) * (t1 @ vr))
    t3 = round_fp16(vc @ t2)
    if trace is not None:
        trace.update(scale=s, vc=vc, vr=vr, rt=rt, t1=t1, t2=t2, t3=t3)
    return (t3 @ vr.T) / (s * lam * lam)


def precond_fp8(Vc, Vr, sc, sr, lam, r, trace=None):
    """FP8-e4m3 chain with 32-entry block scales along each contraction.
    `trace` (a dict, optional) receives every quantised operand as values
    (codes times 2^e): vct = Q(Vc^T), rq = Q(r), t1 = Q(Vc^T R), vr = Q(Vr),
    t2 = Q(S' .* (t1 Vr)), vc = Q(Vc), t3 = Q(Vc t2), vrt = Q(Vr^T), each
    blocked along the contraction of the product it feeds."""
    def left(x):     # contraction over columns (axis 1)
        q, e = quantize_e4m3_blocks(x, axis=1)
        return dequant(q, e, axis=1)

    def right(x):    # contraction over rows (axis 0)
        q, e = quantize_e4m3_blocks(x, axis=0)
        return dequant(q, e, axis=0)

    r = np.asarray(r, dtype=np.float64)
    vct, rq = left(Vc.T), right(r)
    t1 = left(vct @ rq)
    vrq = right(Vr)
    t2 = right(s_prime(sc, sr, lam) * (t1 @ vrq))
    vcq = left(Vc)
    t3 = left(vcq @ t2)
    vrt = right(Vr.T)
    if trace is not None:
        trace.update(vct=vct, rq=rq, t1=t1, vr=vrq, t2=t2, vc=vcq, t3=t3, vrt=vrt)
    return (t3 @ vrt) / (lam * lam)


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


# --------------------------------------------------------------------------
# elementwise bounds for an implementation of the reduced-precision chains
# --------------------------------------------------------------------------
#
# An implementation stores the same operands as the emulations above but
# accumulates each product in FP32 (any order), and rounds each stored
# intermediate from its own FP32 value.  Where that value lies close to a
# rounding boundary of the storage format the two sides can round to
# neighbouring values; after that the difference propagates through the
# remaining products.  The bounds below follow that propagation entry by
# entry: with `acc` the emulation's exact value and E a bound on the
# implementation's distance from it, the implementation's rounded value lies
# in [rnd(acc - E), rnd(acc + E)] (rounding is monotone), so the stored
# entries differ by at most
#     D = max(rnd(acc + E) - rnd(acc), rnd(acc) - rnd(acc - E)),
# which is 0 wherever acc is farther than E from a boundary.  FP32
# accumulation of m products in any order is bounded by gamma_m u32 sum |terms|
# (Higham, Accuracy and Stability of Numerical Algorithms, ch. 3).

U32 = 2.0 ** -24


def _inflate(e):
    """Bound slack for the FP64 arithmetic of the bound itself."""
    return np.asarray(e, dtype=np.float64) * (1.0 + 1e-9) + 1e-300


def _flip_gap(acc, e, rnd):
    """max |rnd(a) - rnd(acc)| over |a - acc| <= e, for monotone rnd."""
    e = _inflate(e)
    mid = rnd(acc)
    return np.maximum(np.abs(rnd(acc + e) - mid), np.abs(mid - rnd(acc - e)))


def fp16_chain_bound(Vc, Vr, sc, sr, lam, r, rnorm=None):
    """Elementwise bound on |z_impl - precond_fp16(...)| for an FP16 chain
    that stores FP16 V rounded from any value within half an FP32 unit of
    the given V (so V may be the FP32 copy of the factor), fp16(scale r)
    and fp16 of its own FP32 intermediates, accumulates in FP32, forms S' in
    FP32 (to within 4 u32 relative of s_prime) and scales the output by the
    FP32 value of 1 / (scale lambda^2)."""
    n = Vc.shape[0]
    r = np.asarray(r, dtype=np.float64)
    if rnorm is None:
        rnorm = float(np.linalg.norm(r))
    s = pow2_scale_for_norm(rnorm)
    g = gamma(n + 8, U32)
    vc, vr = round_fp16(Vc), round_fp16(Vr)
    # the implementation may round V to FP16 from any value within half an
    # FP32 unit of the V given here (its FP64 or its FP32 copy)
    dvc = _flip_gap(np.asarray(Vc, dtype=np.float64), U32 * np.abs(Vc), round_fp16)
    dvr = _flip_gap(np.asarray(Vr, dtype=np.float64), U32 * np.abs(Vr), round_fp16)
    avc, avr = np.abs(vc) + dvc, np.abs(vr) + dvr
    rt = round_fp16(s * r)
    art = np.abs(rt)
    # stage 1: T1 = fp16(Vc^T rt)
    acc1 = vc.T @ rt
    e1 = g * (avc.T @ art) + dvc.T @ art
    t1 = round_fp16(acc1)
    d1 = _flip_gap(acc1, e1, round_fp16)
    # stage 2: T2 = fp16(fl32(S' * (T1 Vr)))
    acc2 = t1 @ vr
    at1 = np.abs(t1) + d1
    e2a = d1 @ avr + np.abs(t1) @ dvr + g * (at1 @ avr)
    sp = s_prime(sc, sr, lam)
    v2 = sp * acc2
    e2 = sp * e2a + 5 * U32 * sp * (np.abs(acc2) + e2a)
    t2 = round_fp16(v2)
    d2 = _flip_gap(v2, e2, round_fp16)
    # stage 3: T3 = fp16(Vc T2)
    acc3 = vc @ t2
    at2 = np.abs(t2) + d2
    e3 = avc @ d2 + dvc @ np.abs(t2) + g * (avc @ at2)
    t3 = round_fp16(acc3)
    d3 = _flip_gap(acc3, e3, round_fp16)
    # stage 4: z = fl32(fl32(T3 Vr^T) * fl32(1 / (scale lambda^2)))
    acc4 = t3 @ vr.T
    at3 = np.abs(t3) + d3
    e4 = d3 @ avr.T + np.abs(t3) @ dvr.T + g * (at3 @ avr.T)
    zs = 1.0 / (s * lam * lam)
    return _inflate(zs * e4 + 3 * U32 * zs * (np.abs(acc4) + e4))


def _block_view(x, axis, block=FP8_BLOCK):
    """x with `axis` moved last and split into (nblocks, block), zero padded."""
    x = np.moveaxis(np.asarray(x, dtype=np.float64), axis, -1)
    k = x.shape[-1]
    nb = (k + block - 1) // block
    xp = np.pad(x, [(0, 0)] * (x.ndim - 1) + [(0, nb * block - k)])
    return xp.reshape(x.shape[:-1] + (nb, block)), k


def _unblock(xb, k, axis):
    x = xb.reshape(xb.shape[:-2] + (-1,))[..., :k]
    return np.moveaxis(x, -1, axis)


def _e4m3_flip_gap(acc, e, axis):
    """Bound on |stored_impl - stored_emul| for one block-quantised e4m3
    operand: the implementation's value of each entry is within e of the
    emulation's `acc`, and it picks each block's exponent from its own
    values.  Candidate exponents are those of every block maximum in
    [max(|acc| - e), max(|acc| + e)]."""
    e = _inflate(e)
    ab, k = _block_view(acc, axis)
    eb_, _ = _block_view(e, axis)
    lo = np.max(np.maximum(np.abs(ab) - eb_, 0.0), axis=-1)
    hi = np.max(np.abs(ab) + eb_, axis=-1)
    ex_emul = block_exponents(_unblock(ab, k, -1), axis=-1)           # (..., nb)
    ex_lo = np.where(lo > 0, block_exponents(lo[..., None], axis=-1)[..., 0], -127)
    ex_hi = block_exponents(hi[..., None], axis=-1)[..., 0]
    ef = ex_emul[..., None].astype(np.float64)
    q_emul = np.exp2(ef) * round_e4m3(ab * np.exp2(-ef))
    gap = np.zeros_like(ab)
    for d in (0, 1):
        ec = np.minimum(ex_lo + d, ex_hi)[..., None].astype(np.float64)
        qa = np.exp2(ec) * round_e4m3((ab + eb_) * np.exp2(-ec))
        qb = np.exp2(ec) * round_e4m3((ab - eb_) * np.exp2(-ec))
        gap = np.maximum(gap, np.maximum(np.abs(qa - q_emul), np.abs(q_emul - qb)))
    # blocks whose maximum could cross more than one power of two (or vanish):
    # every entry of both sides lies within 1/16 of its value plus half the
    # largest subnormal quantum
    wide = ((ex_hi - ex_lo) > 1)[..., None]
    loose = (np.abs(ab) + eb_) * (2.0 + 2.0 ** -3) + np.exp2(ex_hi[..., None] - 9.0)
    gap = np.where(wide, loose, gap)
    return _unblock(gap, k, axis)


def fp8_chain_bound(Vc, Vr, sc, sr, lam, r):
    """Elementwise bound on |z_impl - precond_fp8(Vc, Vr, ...)| for an FP8
    chain that quantises the same FP32 operands (pass FP32-representable
    Vc, Vr and r), accumulates each block-scaled product in FP32, and
    quantises its own FP32 intermediates with exponents from its own block
    maxima (S' in FP32 as for FP16)."""
    n = Vc.shape[0]
    g = gamma(n + 8, U32)
    tr = {}
    precond_fp8(Vc, Vr, sc, sr, lam, r, trace=tr)
    avct, arq = np.abs(tr["vct"]), np.abs(tr["rq"])
    # stage 1: T1 = Q_rows(Vc^T R)
    acc1 = tr["vct"] @ tr["rq"]
    e1 = g * (avct @ arq)
    d1 = _e4m3_flip_gap(acc1, e1, axis=1)
    # stage 2: T2 = Q_cols(S' .* (T1 Vr))
    avr = np.abs(tr["vr"])
    acc2 = tr["t1"] @ tr["vr"]
    e2a = d1 @ avr + g * ((np.abs(tr["t1"]) + d1) @ avr)
    sp = s_prime(sc, sr, lam)
    v2 = sp * acc2
    e2 = sp * e2a + 5 * U32 * sp * (np.abs(acc2) + e2a)
    d2 = _e4m3_flip_gap(v2, e2, axis=0)
    # stage 3: T3 = Q_rows(Vc T2)
    avc = np.abs(tr["vc"])
    acc3 = tr["vc"] @ tr["t2"]
    e3 = avc @ d2 + g * (avc @ (np.abs(tr["t2"]) + d2))
    d3 = _e4m3_flip_gap(acc3, e3, axis=1)
    # stage 4: z = fl32(T3 Vr^T) * fl32(1 / lambda^2)
    avrt = np.abs(tr["vrt"])
    acc4 = tr["t3"] @ tr["vrt"]
    e4 = d3 @ avrt + g * ((np.abs(tr["t3"]) + d3) @ avrt)
    zs = 1.0 / (lam * lam)
    return _inflate(zs * e4 + 3 * U32 * zs * (np.abs(acc4) + e4))
