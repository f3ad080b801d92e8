"""Autotuner: the configuration it returns meets the accuracy target against
the oracle's direct sum (Eq. 1) when re-run from scratch, and its table holds
only candidates that met the target."""
import numpy as np
import pytest

from paper_1110_4876_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_tuned_point_meets_target(orc, prec):
    from gpu_util import Dev, gravity, make_ctx
    from paper_1110_4876_amd import autotune, rb
    from paper_1110_4876_amd.system import System
    from paper_1110_4876_amd.metrics import force_errors
    pr = inputs.sheet(8000, seed=3)
    t_kick = 0.5 * pr.dt
    tg = inputs.sample_targets(pr.n, 512, seed=1)
    p = orc.make_params(**pr.params)
    ref = orc.direct(p, pr.x, pr.y, pr.z, pr.m, n_active=pr.n_active,
                     s=orc.shear_offset(p, t_kick), targets=tg)
    sysm = System(pr)
    precision = rb.RB_FP32_MIXED if prec == "fp32" else rb.RB_FP64
    target = 1e-4
    best = autotune.tune(sysm, ref, tg, t_kick, precision=precision, rms_target=target,
                         leafs=(1, 4), groups=(32, 64), splits=(0, 1), graphs=(0, 1),
                         steps=2, repeats=1)
    assert best["table"], "empty table"
    assert all(r["rms"] <= target for r in best["table"])
    assert best["ms_per_step"] == min(r["ms_per_step"] for r in best["table"])
    # re-run the chosen configuration from scratch
    d = Dev(pr)
    c = make_ctx(pr, precision=precision, theta=best["theta"], leaf_size=best["leaf_size"],
                 group_size=best["group_size"], split_images=best["split_images"],
                 use_graph=best["use_graph"])
    try:
        a = gravity(c, d, pr.n, t_kick)[tg]
    finally:
        rb.rb_destroy(c)
    e = force_errors(a, ref)
    assert e["rms"] <= target, e
    assert np.isclose(e["rms"], best["rms"], rtol=1e-6, atol=0), (e["rms"], best["rms"])


def test_tuned_batch_meets_target():
    # a batch of patches: each sampled target is checked against the direct
    # sum over its own patch (System.direct through the C ABI, FP64)
    from paper_1110_4876_amd import autotune, rb
    from paper_1110_4876_amd.metrics import force_errors
    from paper_1110_4876_amd.system import System
    sysm = System(inputs.batch(6, n_min=1500, n_max=5000, seed0=11))
    t_kick = 0.5 * sysm.dt
    tg = sysm.sample_targets(per_patch=64, seed=2)
    ref = sysm.direct(tg, t_kick)
    best = autotune.tune(sysm, ref, tg, t_kick, precision=rb.RB_FP32_MIXED, rms_target=1e-4,
                         leafs=(1, 2), groups=(16, 32), splits=(0,), graphs=(0, 1), steps=2,
                         repeats=1)
    ctx = sysm.create(rb.RB_FP32_MIXED, theta=best["theta"], leaf_size=best["leaf_size"],
                      group_size=best["group_size"], split_images=best["split_images"])
    try:
        a = sysm.gravity(ctx, t_kick).cpu().numpy()[tg]
    finally:
        rb.rb_destroy(ctx)
    assert force_errors(a, ref)["rms"] <= 1e-4


def test_system_direct_matches_oracle(orc):
    # the benchmark's reference (GPU direct sum per patch) against the oracle
    from paper_1110_4876_amd.system import System
    probs = inputs.batch(3, n_min=1000, n_max=3000, seed0=5)
    sysm = System(probs)
    t = 777.0
    tg = sysm.sample_targets(per_patch=40, seed=1)
    got = sysm.direct(tg, t)
    for k, pr in enumerate(probs):
        lo, hi = sysm.offsets[k], sysm.offsets[k + 1]
        sel = (tg >= lo) & (tg < hi)
        p = orc.make_params(**pr.params)
        ref = orc.direct(p, pr.x, pr.y, pr.z, pr.m, n_active=pr.n,
                         s=orc.shear_offset(p, t), targets=tg[sel] - lo)
        err = np.sqrt(np.sum((got[sel] - ref) ** 2) / np.sum(ref ** 2))
        assert err <= 1e-13, (k, err)
