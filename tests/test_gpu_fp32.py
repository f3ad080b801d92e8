"""FP32-mixed grouped walk: gated against the FP64 direct sum (Eq. 1), and
against the FP64 per-particle walk at theta = 0 (precision-only error)."""
import numpy as np
import pytest

from paper_1110_4876_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("group", [64, 32, 16])
def test_theta_zero_precision_only(group):
    # theta = 0: every term is a particle term, so the FP32 walk differs from
    # the FP64 walk only by FP32 rounding of group-relative coordinates
    from gpu_util import Dev, gravity, make_ctx, rms_rel
    from paper_1110_4876_amd import rb
    for pr, t in ((inputs.sheet(6000, seed=1).with_params(theta=0.0), 300.0),
                  (inputs.plummer(6000, seed=2, b=0.01).with_params(theta=0.0), 0.0)):
        d = Dev(pr, with_v=False)
        c64 = make_ctx(pr)
        c32 = make_ctx(pr, precision=rb.RB_FP32_MIXED, group_size=group)
        try:
            ref = gravity(c64, d, pr.n, t)
            a = gravity(c32, d, pr.n, t)
        finally:
            rb.rb_destroy(c64)
            rb.rb_destroy(c32)
        # FP32 unit roundoff 6e-8 per term, amplified by the cancellation of
        # in-plane forces (sum |a_j| / |sum a_j| ~ 10-100 in the sheet)
        assert rms_rel(a, ref) <= 1e-5, rms_rel(a, ref)
