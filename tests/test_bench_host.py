"""Host-side pieces of bench.py that need no GPU: the smooth FFT sizes and
the zero-padded FFT form of H p that the matvec sweep times against the
direct blurs, checked against the oracle's normal operator."""
import numpy as np
import pytest

import bench
import synthetic as S
from oracle import solvers as SV


def test_smooth_size():
    for m in (1, 7, 11, 1031, 1047, 1055, 2048):
        L = bench.smooth_size(m)
        assert L >= m
        r = L
        for f in (2, 3, 5, 7):
            while r % f == 0:
                r //= f
        assert r == 1
        # nothing smaller qualifies
        for q in range(m, L):
            r = q
            for f in (2, 3, 5, 7):
                while r % f == 0:
                    r //= f
            assert r != 1


@pytest.mark.parametrize("n,k,pad", [(40, 15, 0), (33, 9, 0), (32, 15, 5)])
def test_fft_normal_equals_oracle(n, k, pad):
    """The FFT form at the smallest admissible L = n + h (and a larger one)
    equals the oracle's A^T A p."""
    torch = pytest.importorskip("torch")
    h = (k - 1) // 2
    psf = S.psf_moffat_motion(k, 3.0, 2.5, 4.0, 0.6)
    p = np.random.default_rng(n + k).standard_normal((n, n))
    L = n + h + pad
    pf = bench.psf_spectrum(psf, L, "cpu").to(torch.complex128)
    got = bench.fft_normal(torch.from_numpy(p), pf, pf.conj(), L, h).numpy()
    ref = SV.NormalOperator(psf, n, 0.0, use_fft=False).H(p)
    # the spectrum is of the FP32-rounded PSF
    assert np.abs(got - ref).max() <= 1e-6 * np.abs(ref).max()


def test_fft_normal_bytes_counts_each_pass():
    """Algorithmic bytes of one H p by the five FFT passes, counted pass by
    pass: rows_fwd reads p (4 n^2) and writes the half spectra S (8 F n);
    each column pass reads its F lines (8 F n) and the PSF spectrum (8 F L)
    and writes T (8 F n); rows_mid reads T and writes S (8 F n each);
    rows_out reads T (8 F n) and p (4 n^2) and writes w (4 n^2)."""
    for n, L in ((1024, 1080), (2048, 2100), (100, 128)):
        F = L // 2 + 1
        per_pass = [4 * n * n + 8 * F * n,
                    8 * F * n + 8 * F * L + 8 * F * n,
                    8 * F * n + 8 * F * n,
                    8 * F * n + 8 * F * L + 8 * F * n,
                    8 * F * n + 4 * n * n + 4 * n * n]
        assert bench.fft_normal_bytes(n, L) == sum(per_pass)
    assert bench.fft_normal_bytes(1024, 1080) == 57386368
