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
