"""What the trained lambda network gains over the method without it.

The network is trained on the GPU by the library's own kernels on generated
256 x 256 problems (2048: 1024 PSFs x 2 images; the full workload is
20,000 problems, see paper_2311_15393_amd/train_lambda.py), with
optimal-error targets in the KP-SVD basis.  On held-out problems of the
uneven batch (sizes 128..1024, never seen in training) its lambda, with GCV
as the fallback judge, is compared with the KP-GCV grid choice: distance to
the optimal-error lambda, and the relative error of the FP16-KP FPCG
solution against the true image."""
import numpy as np
import pytest

from tests.gpu_util import require_gpu, say

pytestmark = pytest.mark.gpu


def test_learned_lambda_beats_gcv():
    require_gpu()
    from paper_2311_15393_amd.train_lambda import run
    _, out = run(groups=1024, per_psf=2, epochs=150, ntest=32, val_groups=48,
                 log=lambda m: say(m))
    say(f"gain summary: {out}")
    # the network generalises: held-out error well below GCV's
    assert out["rmse_val"] < 0.6 * out["rmse_val_gcv"]
    assert out["rmse_test_net"] < out["rmse_test_gcv"]
    # and the solutions are closer to the true images on average, with no
    # problem made much worse (GCV's fallback catches bad predictions)
    assert out["err_learned"] < out["err_gcv"]
    assert out["wins"] >= out["test_problems"] // 2
    assert out["worst_ratio"] < 1.25
