"""Pins for the reduced-precision formats and emulated preconditioner chains."""
import math
import struct

import numpy as np
import pytest
import torch

import synthetic as S
from oracle import kp as KP
from oracle import quant as Q


def test_e4m3_codes_match_library_table():
    """All 256 e4m3 codes decoded from the format definition equal an
    independent library's decoding of the same bytes."""
    codes = torch.arange(256, dtype=torch.uint8)
    lib = codes.view(torch.float8_e4m3fn).to(torch.float64).numpy()
    mine = np.array([Q.e4m3_decode(c) for c in range(256)])
    nan = np.isnan(lib)
    assert np.array_equal(nan, np.isnan(mine))
    assert np.array_equal(lib[~nan], mine[~nan])
    assert np.nanmax(mine) == 448.0 and np.nanmin(np.abs(mine[mine != 0])) == 2.0 ** -9


def test_e4m3_rounding_matches_library_cast():
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.standard_normal(20000) * 10.0,
        rng.uniform(-448, 448, 20000),
        rng.uniform(-0.02, 0.02, 20000),         # subnormal range
        np.array([0.0, -0.0, 448.0, -448.0, 2 ** -10, 3 * 2 ** -10, 0.01953125]),
    ])
    # exact midpoints between neighbouring codes test ties-to-even
    vals = np.array(sorted({Q.e4m3_decode(c) for c in range(127)}))
    mids = 0.5 * (vals[1:] + vals[:-1])
    x = np.concatenate([x, mids, -mids])
    lib = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(Q.round_e4m3(x), lib)


def test_e4m3_saturates():
    assert Q.round_e4m3(np.array([1000.0, -1e9]))[0] == 448.0
    assert Q.round_e4m3(np.array([-1e9]))[0] == -448.0


def test_pow2_scale():
    for v in [1e-30, 3.7e-7, 1.0, 16384.0, 16385.0, 5e20]:
        s = Q.pow2_scale_for_norm(v)
        assert math.frexp(s)[0] == 0.5          # a power of two
        assert 2.0 ** 13 <= s * v < 2.0 ** 14


def test_block_exponents_are_tight():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((5, 100)) * np.exp(rng.uniform(-20, 20, (5, 1)))
    x[2, 32:64] = 0.0
    e = Q.block_exponents(x, axis=1)
    assert e.shape == (5, 4)
    for i in range(5):
        for b in range(4):
            blk = np.abs(x[i, 32 * b:32 * b + 32])
            if blk.max() == 0:
                assert e[i, b] == -127
                continue
            scaled = blk.max() * 2.0 ** -e[i, b]
            assert 224.0 < scaled <= 448.0


def _factors(n, lam=0.01):
    psf = S.psf_gaussian(15, 3.0, 1.5, 0.5)
    kp = KP.kp_svd(psf, n)
    r = np.random.default_rng(2).standard_normal((n, n))
    return kp, r, lam


def test_fp16_chain_accuracy_and_range():
    """The FP16 chain is an O(u16) perturbation of the exact solve, and its
    scaling keeps every intermediate inside FP16's range."""
    kp, r, lam = _factors(64)
    z = KP.precond_solve(kp, lam, r)
    z16 = Q.precond_fp16(kp.Vc, kp.Vr, kp.sc, kp.sr, lam, r)
    rel = np.linalg.norm(z16 - z) / np.linalg.norm(z)
    assert 1e-5 < rel < 2e-2
    s = Q.pow2_scale_for_norm(np.linalg.norm(r))
    assert np.abs(s * r).max() < Q.FP16_MAX


def test_fp8_chain_accuracy():
    kp, r, lam = _factors(64)
    z = KP.precond_solve(kp, lam, r)
    z8 = Q.precond_fp8(kp.Vc, kp.Vr, kp.sc, kp.sr, lam, r)
    rel = np.linalg.norm(z8 - z) / np.linalg.norm(z)
    assert 1e-3 < rel < 0.2


def test_fp32_chain_bound_holds_for_float32_arithmetic():
    """The first-order accumulation bound covers an actual float32 chain
    (numpy float32 matmul: FP32 products and sums)."""
    kp, r, lam = _factors(96)
    f = np.float32
    vc, vr = kp.Vc.astype(f), kp.Vr.astype(f)
    sp = Q.s_prime(kp.sc, kp.sr, lam).astype(f)
    t = (vc.T @ r.astype(f)) @ vr
    z32 = ((vc @ (sp * t)) @ vr.T).astype(np.float64) / (lam * lam)
    ref = Q.precond_fp32(kp.Vc, kp.Vr, kp.sc, kp.sr, lam, r)
    bound = Q.fp32_chain_bound(kp.Vc, kp.Vr, kp.sc, kp.sr, lam, r)
    assert np.all(np.abs(z32 - ref) <= bound)
    assert np.abs(z32 - ref).max() > 0


# --------------------------------------------------------------------------
# pins of the emulated chains against values fixed by exact arithmetic and
# by hand, independent of the emulation's own formulas
# --------------------------------------------------------------------------

def _signed_perm(rng, n):
    m = np.zeros((n, n))
    m[np.arange(n), rng.permutation(n)] = rng.choice([-1.0, 1.0], n)
    return m


def _exact_case(n=40, seed=0):
    """Factors whose products are exact in every format: V_c, V_r signed
    permutations; S' in {1, 1/2} (s_c[i] s_r[j] in {0, lambda}, lambda = 1/2,
    with a row pattern unlike the column pattern, so S' and its transpose
    differ); r with entries of two significant bits spread over 2^-6 .. 2^3
    (exact in FP16 after any power-of-two scale, and in e4m3 under a
    32-entry block scale since each block spans less than 2^8)."""
    rng = np.random.default_rng(seed)
    lam = 0.5
    sc = np.where(rng.uniform(size=n) < 0.5, 0.5, 0.0)
    sr = np.where(np.arange(n) % 3 == 0, 1.0, 0.0)
    vc, vr = _signed_perm(rng, n), _signed_perm(rng, n)
    r = rng.choice([-1.0, 1.0], (n, n)) * rng.choice([1.0, 1.5], (n, n)) \
        * np.exp2(rng.integers(-6, 4, (n, n)))
    kp = KP.KPSVD(n=n, Ac=None, Ar=None, Uc=None, sc=sc, Vc=vc, Ur=None, sr=sr, Vr=vr,
                  s_psf=None)
    return kp, r, lam


def test_fp16_chain_exact_products_equal_fp64_solve():
    """With exact products every FP16 rounding is the identity, so the chain
    (scale, S' folding, lambda^2 restored at the end) must equal the FP64
    preconditioner solve of eq. (PreconSolve) bit for bit."""
    kp, r, lam = _exact_case()
    z = KP.precond_solve(kp, lam, r)
    z16 = Q.precond_fp16(kp.Vc, kp.Vr, kp.sc, kp.sr, lam, r)
    assert np.array_equal(z16, z)
    # the case can tell S' from its transpose and Vc from Vr
    sp = Q.s_prime(kp.sc, kp.sr, lam)
    assert not np.array_equal(sp, sp.T)
    assert not np.array_equal(
        Q.precond_fp16(kp.Vr, kp.Vc, kp.sc, kp.sr, lam, r), z)


def test_fp8_chain_exact_products_equal_fp64_solve():
    """The same exact-product case through the block-scaled e4m3 chain."""
    kp, r, lam = _exact_case(seed=1)
    z = KP.precond_solve(kp, lam, r)
    z8 = Q.precond_fp8(kp.Vc, kp.Vr, kp.sc, kp.sr, lam, r)
    assert np.array_equal(z8, z)


def test_fp16_chain_hand_worked_ties():
    """A 2 x 2 case worked by hand, whose scaled residual and intermediates
    land on FP16 ties (round half to even) at every stored stage.

    lambda = 1/4 (lambda^2 = 2^-4), s_c = (1/2, 0), s_r = (1/2, 1/2):
    S' = lambda^2 / (s_c^2 s_r^2 + lambda^2) = [[1/2, 1/2], [1, 1]].
    V_c = V_r = [[1, 1], [0, 1]] (the chain is plain arithmetic; V need not
    be orthogonal for this check).
    r = [[1 + 2^-11, 3 * 2^-38], [2052 * 2^-13, 2^-11]], ||r|| = 1.031...,
    so the scale is 2^13 (||scale r|| in [2^13, 2^14)).
      scale r = [[8196, 1.5 * 2^-24], [2052, 4]]
        8196 lies halfway between 8192 and 8200 (spacing 8): even -> 8192;
        1.5 * 2^-24 halfway between the subnormals 2^-24 and 2^-23: -> 2^-23
        (with a scale of 2^14 it would be 3 * 2^-24, exact)
      rt = [[8192, 2^-23], [2052, 4]]
      V_c^T rt = [[8192, 2^-23], [10244, 4 + 2^-23]]
        10244 halfway between 10240 and 10248: even -> 10240; 4 + 2^-23 -> 4
      t1 = [[8192, 2^-23], [10240, 4]]
      t1 V_r = [[8192, 8192 + 2^-23], [10240, 10244]]
      S' .* that = [[4096, 4096 + 2^-24], [10240, 10244]] -> 10244 -> 10240
      t2 = [[4096, 4096], [10240, 10240]]
      t3 = V_c t2 = [[14336, 14336], [10240, 10240]] (exact)
      t3 V_r^T = [[28672, 14336], [20480, 10240]]
      z = that / (2^13 * 2^-4) = [[56, 28], [40, 20]]."""
    lam = 0.25
    sc = np.array([0.5, 0.0])
    sr = np.array([0.5, 0.5])
    v = np.array([[1.0, 1.0], [0.0, 1.0]])
    r = np.array([[1.0 + 2.0 ** -11, 3.0 * 2.0 ** -38],
                  [2052.0 * 2.0 ** -13, 2.0 ** -11]])
    tr = {}
    z = Q.precond_fp16(v, v, sc, sr, lam, r, trace=tr)
    assert tr["scale"] == 2.0 ** 13
    assert np.array_equal(tr["rt"], [[8192.0, 2.0 ** -23], [2052.0, 4.0]])
    assert np.array_equal(tr["t1"], [[8192.0, 2.0 ** -23], [10240.0, 4.0]])
    assert np.array_equal(tr["t2"], [[4096.0, 4096.0], [10240.0, 10240.0]])
    assert np.array_equal(tr["t3"], [[14336.0, 14336.0], [10240.0, 10240.0]])
    assert np.array_equal(z, [[56.0, 28.0], [40.0, 20.0]])


def _e4m3_grid():
    """Non-negative finite e4m3 values with their codes, decoded by an
    independent library (torch's float8_e4m3fn)."""
    codes = torch.arange(0, 127, dtype=torch.uint8)
    vals = codes.view(torch.float8_e4m3fn).to(torch.float64).numpy()
    return vals, codes.numpy().astype(int)


def _quantize_loop(x, axis):
    """Block quantisation written entry by entry from the definitions: the
    block is the run of 32 consecutive entries along `axis` holding the
    entry; its exponent is the smallest integer e with max|block| 2^-e <=
    448, found by stepping e; the scaled entry goes to the nearest e4m3 value
    (ties: the one with the even code)."""
    vals, codes = _e4m3_grid()
    out = np.zeros_like(x)
    rows, cols = x.shape
    for i in range(rows):
        for j in range(cols):
            if axis == 0:
                b0 = (i // 32) * 32
                blk = x[b0:min(b0 + 32, rows), j]
            else:
                b0 = (j // 32) * 32
                blk = x[i, b0:min(b0 + 32, cols)]
            amax = np.max(np.abs(blk))
            if amax == 0.0:
                continue
            e = int(np.floor(np.log2(amax))) - 12
            while amax * 2.0 ** -e > 448.0:
                e += 1
            y = abs(x[i, j]) * 2.0 ** -e
            d = np.abs(vals - y)
            best = np.flatnonzero(d == d.min())
            pick = best[0] if len(best) == 1 else best[codes[best] % 2 == 0][0]
            out[i, j] = np.copysign(vals[pick] * 2.0 ** e, x[i, j])
    return out


def test_e4m3_block_quantisation_matches_entrywise_loop():
    """quantize_e4m3_blocks / dequant against the entry-by-entry loop, on a
    40 x 70 matrix (ragged last blocks on both axes) whose magnitudes vary
    by row and by column, so blocking along the wrong axis changes the
    result; values include exact e4m3 ties."""
    rng = np.random.default_rng(5)
    x = rng.standard_normal((40, 70)) * np.exp2(rng.integers(-12, 12, (40, 1))) \
        * np.exp2(rng.integers(-6, 6, (1, 70)))
    x[3, 5] = 0.0
    x[7, :] = 0.0                                     # a zero row: zero blocks along axis 1
    x[10, 40] = x[10, 32:64].max() * (1 + 1 / 16) if x[10, 32:64].max() > 0 else 1.0
    ref = {}
    for axis in (0, 1):
        q, e = Q.quantize_e4m3_blocks(x, axis=axis)
        got = Q.dequant(q, e, axis=axis)
        ref[axis] = _quantize_loop(x, axis)
        assert np.array_equal(got, ref[axis]), axis
    assert not np.array_equal(ref[0], ref[1])


def test_fp8_chain_stages_match_entrywise_quantisation():
    """Each stored operand of the FP8 chain equals the entry-by-entry
    quantisation (blocked along the contraction it feeds) of the exact
    product of the previous stored operands, on a ragged 40 x 40 case."""
    rng = np.random.default_rng(8)
    n = 40
    vc = np.linalg.qr(rng.standard_normal((n, n)))[0]
    vr = np.linalg.qr(rng.standard_normal((n, n)))[0]
    sc, sr, lam = np.sort(rng.uniform(0, 1, n))[::-1], np.sort(rng.uniform(0, 1, n))[::-1], 0.05
    r = rng.standard_normal((n, n)) * np.exp2(rng.integers(-8, 8, (n, 1)))
    tr = {}
    z = Q.precond_fp8(vc, vr, sc, sr, lam, r, trace=tr)
    assert np.array_equal(tr["vct"], _quantize_loop(vc.T, 1))
    assert np.array_equal(tr["rq"], _quantize_loop(r, 0))
    assert np.array_equal(tr["t1"], _quantize_loop(tr["vct"] @ tr["rq"], 1))
    assert np.array_equal(tr["vr"], _quantize_loop(vr, 0))
    sp = Q.s_prime(sc, sr, lam)
    assert np.array_equal(tr["t2"], _quantize_loop(sp * (tr["t1"] @ tr["vr"]), 0))
    assert np.array_equal(tr["vc"], _quantize_loop(vc, 1))
    assert np.array_equal(tr["t3"], _quantize_loop(tr["vc"] @ tr["t2"], 1))
    assert np.array_equal(tr["vrt"], _quantize_loop(vr.T, 0))
    assert np.array_equal(z, (tr["t3"] @ tr["vrt"]) / (lam * lam))


def test_fp16_chain_stages_match_library_half_casts():
    """Each stored operand of the FP16 chain equals CPython's binary16
    packing (struct format 'e': IEEE half, round half to even, straight from
    the double) of the exact product of the previous stored operands, on a
    48 x 48 case with a residual spanning 2^-30."""
    rng = np.random.default_rng(9)
    n = 48
    vc = np.linalg.qr(rng.standard_normal((n, n)))[0]
    vr = np.linalg.qr(rng.standard_normal((n, n)))[0]
    sc, sr, lam = np.sort(rng.uniform(0, 1, n))[::-1], np.sort(rng.uniform(0, 1, n))[::-1], 0.01
    r = rng.standard_normal((n, n)) * np.exp2(rng.integers(-30, 0, (n, n)))

    def h(a):
        a = np.asarray(a, dtype=np.float64)
        flat = [struct.unpack("<e", struct.pack("<e", float(v)))[0] for v in a.ravel()]
        return np.array(flat).reshape(a.shape)

    tr = {}
    z = Q.precond_fp16(vc, vr, sc, sr, lam, r, trace=tr)
    nrm = np.linalg.norm(r)
    assert 2.0 ** 13 <= tr["scale"] * nrm < 2.0 ** 14
    assert np.array_equal(tr["rt"], h(tr["scale"] * r))
    assert np.array_equal(tr["t1"], h(h(vc).T @ tr["rt"]))
    sp = (np.float32(lam * lam) / (np.float32(sc ** 2)[:, None] * np.float32(sr ** 2)[None, :]
                                   + np.float32(lam * lam))).astype(np.float64)
    assert np.array_equal(tr["t2"], h(sp * (tr["t1"] @ h(vr))))
    assert np.array_equal(tr["t3"], h(h(vc) @ tr["t2"]))
    assert np.array_equal(z, (tr["t3"] @ h(vr).T) / (tr["scale"] * lam * lam))


def _fp32_impl_fp16(vc, vr, sc, sr, lam, r):
    """An FP16 chain as an implementation runs it: FP16 operands, float32
    matrix products (FP32 accumulation), each intermediate rounded from its
    FP32 value."""
    f, hf = np.float32, np.float16
    s = Q.pow2_scale_for_norm(np.linalg.norm(r))
    v16c, v16r = vc.astype(hf).astype(f), vr.astype(hf).astype(f)
    rt = (s * r).astype(hf).astype(f)
    t1 = (v16c.T @ rt).astype(hf).astype(f)
    sp = Q.s_prime(sc, sr, lam).astype(f)
    t2 = (sp * (t1 @ v16r)).astype(hf).astype(f)
    t3 = (v16c @ t2).astype(hf).astype(f)
    return ((t3 @ v16r.T) * f(1.0 / (s * lam * lam))).astype(np.float64)


def _fp32_impl_fp8(vc, vr, sc, sr, lam, r):
    """The FP8 chain with float32 products, quantising its own FP32
    intermediates (exponents from its own block maxima)."""
    f = np.float32

    def left(x):
        q, e = Q.quantize_e4m3_blocks(np.asarray(x, dtype=np.float64), axis=1)
        return Q.dequant(q, e, axis=1).astype(f)

    def right(x):
        q, e = Q.quantize_e4m3_blocks(np.asarray(x, dtype=np.float64), axis=0)
        return Q.dequant(q, e, axis=0).astype(f)

    t1 = left(left(vc.T) @ right(r))
    t2 = right(Q.s_prime(sc, sr, lam).astype(f) * (t1 @ right(vr)))
    t3 = left(left(vc) @ t2)
    return ((t3 @ right(vr.T)) * f(1.0 / (lam * lam))).astype(np.float64)


@pytest.mark.parametrize("n", [64, 200])
def test_lowp_chain_bounds_cover_float32_implementations(n):
    """The elementwise bounds on |z_impl - z_emul| hold for chains computed
    with float32 products, where the implementation differs from the
    emulation.  They are worst-case bounds: at n = 64 they stay far below
    |z| (an O(1) mistake such as a swapped factor breaks them), while at
    larger n the sqrt(n) ratio between |V|^T |R| and |V^T R| lets the FP32
    accumulation bound reach FP16's half unit and they grow loose."""
    rng = np.random.default_rng(n)
    psf = S.psf_moffat_motion(15, 4.0, 2.5, 5.0, 0.7)
    kp = KP.kp_svd(psf, n)
    vc, vr = Q.round_fp32(kp.Vc), Q.round_fp32(kp.Vr)
    r = Q.round_fp32(rng.standard_normal((n, n)) * 1e-3)
    lam = 0.01
    exact = Q.precond_fp32(vc, vr, kp.sc, kp.sr, lam, r)
    for impl, emul, bound in (
            (_fp32_impl_fp16, Q.precond_fp16, Q.fp16_chain_bound),
            (_fp32_impl_fp8, Q.precond_fp8, Q.fp8_chain_bound)):
        zi = impl(vc, vr, kp.sc, kp.sr, lam, r)
        ze = emul(vc, vr, kp.sc, kp.sr, lam, r)
        b = bound(vc, vr, kp.sc, kp.sr, lam, r)
        assert np.all(np.abs(zi - ze) <= b), impl.__name__
        assert np.abs(zi - ze).max() > 0
        if n == 64:
            assert np.median(b) < 0.1 * np.median(np.abs(exact)), impl.__name__
            swapped = impl(vr, vc, kp.sc, kp.sr, lam, r)
            assert np.any(np.abs(swapped - ze) > b), impl.__name__
