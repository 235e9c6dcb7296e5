"""Pins for the reduced-precision formats and emulated preconditioner chains."""
import math

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
