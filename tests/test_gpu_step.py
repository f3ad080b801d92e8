"""GPU drift-kick-drift steps against the oracle's step (Sect. 3): leap-frog
with open boundaries, epicycle drift with shear-periodic boundaries, removal
of escaping particles, and checkpoint / resume."""
import os
import tempfile

import numpy as np
import pytest

from paper_1110_4876_amd import inputs

pytestmark = pytest.mark.gpu


def _run_gpu(pr, t, dt, nsteps, **kw):
    from gpu_util import Dev, make_ctx
    from paper_1110_4876_amd import rb
    ctx = make_ctx(pr, **kw)
    try:
        d = Dev(pr)
        rb.rb_step(ctx, d.parts, d.n, pr.n_active, t, dt, nsteps)
        rb.rb_sync(ctx)
        return d.state()
    finally:
        rb.rb_destroy(ctx)


def _close(a, b, rtol, atol=0.0):
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        np.testing.assert_allclose(a[k], b[k], rtol=rtol, atol=atol, err_msg=k)


def test_c0_one_step_matches_oracle(orc):
    pr = inputs.plummer(1024, seed=0)
    p = orc.make_params(**pr.params)
    ref = orc.step(p, pr.state(), pr.m, 0.0, pr.dt, 1, use_tree=True)
    got = _run_gpu(pr, 0.0, pr.dt, 1)
    # positions after the first drift are bit-identical; the kick differs by
    # the walk's summation order only (~1e-16 relative of a dt-sized change)
    _close(got, ref, rtol=1e-14, atol=1e-16)


def test_sheet_one_step_matches_oracle(orc):
    pr = inputs.sheet(4000, seed=3)
    p = orc.make_params(**pr.params)
    t0 = 1000.0
    ref = orc.step(p, pr.state(), pr.m, t0, pr.dt, 1, use_tree=True)
    got = _run_gpu(pr, t0, pr.dt, 1)
    W = pr.params["W"]
    for k in ("x", "y", "z"):
        np.testing.assert_allclose(got[k], ref[k], rtol=0, atol=1e-12 * W, err_msg=k)
    for k in ("vx", "vy", "vz"):
        np.testing.assert_allclose(got[k], ref[k], rtol=0, atol=1e-12, err_msg=k)


def test_drift_only_is_bitwise(orc):
    # G = 0: no kick, the step is two drifts and boundaries -- bit-identical
    for pr in (inputs.plummer(3000, seed=1).with_params(G=0.0),
               inputs.sheet(3000, seed=2).with_params(G=0.0)):
        p = orc.make_params(**pr.params)
        ref = orc.step(p, pr.state(), pr.m, 250.0, pr.dt, 3, use_tree=True)
        got = _run_gpu(pr, 250.0, pr.dt, 3)
        for k in ref:
            np.testing.assert_array_equal(got[k], ref[k], err_msg=k)


def test_multi_step_tracks_oracle(orc):
    pr = inputs.plummer(2000, seed=2, b=0.05)
    p = orc.make_params(**pr.params)
    ref = orc.step(p, pr.state(), pr.m, 0.0, pr.dt, 20, use_tree=True)
    got = _run_gpu(pr, 0.0, pr.dt, 20)
    _close(got, ref, rtol=1e-11, atol=1e-13)


def test_shear_wrap_across_steps(orc):
    # particles pushed across the x faces during the step are re-entered with
    # the shear offset and velocity jump
    pr = inputs.sheet(3000, seed=5)
    W, om = pr.params["W"], pr.params["omega"]
    pr.vx[:200] = np.sign(pr.x[:200]) * 0.5 * W / pr.dt  # cross within a step
    pr.vy[:200] = -1.5 * om * pr.x[:200]
    p = orc.make_params(**pr.params)
    ref = orc.step(p, pr.state(), pr.m, 0.0, pr.dt, 2, use_tree=True)
    got = _run_gpu(pr, 0.0, pr.dt, 2)
    for k in ("x", "y", "z"):
        np.testing.assert_allclose(got[k], ref[k], rtol=0, atol=1e-9 * W, err_msg=k)


def test_escaping_particles_are_removed(orc):
    pr = inputs.plummer(1000, seed=6)
    pr.vx[:3] = 1e6  # leave the root box in the first drift
    p = orc.make_params(**pr.params)
    ref = orc.step(p, pr.state(), pr.m, 0.0, pr.dt, 2, use_tree=True)
    got = _run_gpu(pr, 0.0, pr.dt, 2)
    assert np.all(np.isnan(got["x"][:3])) and np.all(got["vx"][:3] == 0)
    assert np.all(np.isnan(ref["x"][:3]))
    _close({k: v[3:] for k, v in got.items()}, {k: v[3:] for k, v in ref.items()},
           rtol=1e-13, atol=1e-15)


def test_checkpoint_resume_is_bitwise():
    from gpu_util import Dev, make_ctx
    from paper_1110_4876_amd import rb
    pr = inputs.sheet(6000, seed=7)
    ctx = make_ctx(pr)
    try:
        # reference: two calls of 3 steps without a checkpoint in between
        a = Dev(pr)
        rb.rb_step(ctx, a.parts, a.n, a.n, 0.0, pr.dt, 3)
        rb.rb_step(ctx, a.parts, a.n, a.n, 3 * pr.dt, pr.dt, 3)
        rb.rb_sync(ctx)
        b = Dev(pr)
        rb.rb_step(ctx, b.parts, b.n, b.n, 0.0, pr.dt, 3)
        with tempfile.TemporaryDirectory() as td:
            path = os.path.join(td, "state.bin")
            rb.rb_state_save(ctx, b.parts, b.n, 3 * pr.dt, path)
            c = Dev(inputs.sheet(6000, seed=99))
            t = rb.rb_state_load(ctx, c.parts, c.n, path)
            assert t == 3 * pr.dt
            with pytest.raises(rb.RBError):
                rb.rb_state_load(ctx, c.parts, c.n + 1, path)
        rb.rb_step(ctx, c.parts, c.n, c.n, t, pr.dt, 3)
        rb.rb_sync(ctx)
        sa, sc = a.state(), c.state()
    finally:
        rb.rb_destroy(ctx)
    for k in sa:
        np.testing.assert_array_equal(sa[k], sc[k], err_msg=k)


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replay_equals_eager(precision):
    # the step captured once as a HIP graph and replayed: every replay (with
    # eager work and synchronisations in between) matches eager launches
    from gpu_util import Dev, gravity, make_ctx
    from paper_1110_4876_amd import rb
    pr = inputs.sheet(7000, seed=8)
    ce = make_ctx(pr, precision=precision)
    cg = make_ctx(pr, precision=precision, use_graph=1)
    try:
        a, b = Dev(pr), Dev(pr)
        for call in range(3):
            t0 = call * 4 * pr.dt
            rb.rb_step(ce, a.parts, a.n, a.n, t0, pr.dt, 4)
            rb.rb_step(cg, b.parts, b.n, b.n, t0, pr.dt, 4)
            rb.rb_sync(ce)
            rb.rb_sync(cg)
            gravity(ce, Dev(pr, with_v=False), pr.n)  # eager work in between
            sa, sb = a.state(), b.state()
            for k in sa:
                np.testing.assert_array_equal(sa[k], sb[k], err_msg=f"call {call} {k}")
    finally:
        rb.rb_destroy(ce)
        rb.rb_destroy(cg)


def test_phase_timers_across_calls():
    # profile bit 0: nested phase timers (total around the others) stay
    # balanced over several calls with rb_stats in between
    from gpu_util import Dev, make_ctx
    from paper_1110_4876_amd import rb
    pr = inputs.sheet(3000, seed=8)
    ctx = make_ctx(pr, profile=1)
    try:
        d = Dev(pr)
        for call in range(4):
            rb.rb_step(ctx, d.parts, d.n, d.n, 0.0, pr.dt, 3)
            rb.rb_sync(ctx)
            s = rb.rb_stats(ctx)
            assert s["calls"]["walk"] == 3 and s["calls"]["total"] == 1, (call, s["calls"])
            assert s["ms"]["total"] >= s["ms"]["walk"] > 0
    finally:
        rb.rb_destroy(ctx)


def test_periodic_wrap_across_steps(orc):
    # plain periodic boundaries: particles pushed across the x and y faces
    # during the step re-enter through the opposite face, as in the oracle
    pr = inputs.sheet(3000, seed=9).with_params(boundary=inputs.PERIODIC)
    W = pr.params["W"]
    pr.vx[:150] = np.sign(pr.x[:150]) * 0.5 * W / pr.dt
    pr.vy[150:300] = np.sign(pr.y[150:300]) * 0.5 * W / pr.dt
    p = orc.make_params(**pr.params)
    ref = orc.step(p, pr.state(), pr.m, 0.0, pr.dt, 2, use_tree=True)
    got = _run_gpu(pr, 0.0, pr.dt, 2)
    for k in ("x", "y", "z"):
        np.testing.assert_allclose(got[k], ref[k], rtol=0, atol=1e-9 * W, err_msg=k)
    for k in ("vx", "vy", "vz"):
        np.testing.assert_allclose(got[k], ref[k], rtol=1e-9, atol=1e-12, err_msg=k)
