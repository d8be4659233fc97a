"""Autotuner: leaves the run's state untouched, caches its choice, and the
cached tiling gives bitwise the same evolution as any other tiling."""
import json

import numpy as np
import pytest

from paper_1710_10420_amd.inputs import uniform_field
from tests.gpu_util import gpu_prs, gpu_run, host, params_pair, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [(512, 384), (96, 40, 30)])
def test_autotune_preserves_state_and_caches(tmp_path, shape):
    say("autotune", shape)
    prs = gpu_prs()
    deta = 0.25 if len(shape) == 2 else 0.2
    gp, _ = params_pair(shape, deta, m=1.0, W0=10.0, diag_every=5)
    phi0 = uniform_field(shape, 3)
    sim = prs.Sim(gp, phi0=to_dev(phi0))
    sim.step_n(7)
    before = [host(t).copy() for t in sim.state()]
    cache = str(tmp_path / "tune.json")
    us = prs.prs_autotune(sim.ctx, cache, prs.PRS_TUNE_FORCE)
    assert us > 0
    after = [host(t) for t in sim.state()]
    np.testing.assert_array_equal(before[0], after[0])
    np.testing.assert_array_equal(before[1], after[1])
    assert sim.step == 7
    chosen = sim.tiling()
    entries = json.load(open(cache))
    assert len(entries) == 1
    (key, val), = entries.items()
    assert (val["vec"], val["rows"], val["ty"]) == chosen
    assert prs.prs_tuned_tiling(gp, cache) == chosen
    # cached: applied without timing on a fresh context
    sim2 = prs.Sim(gp, phi0=to_dev(phi0))
    prs.prs_autotune(sim2.ctx, cache, 0)
    assert sim2.tiling() == chosen
    # the tuned run continues exactly like a run with the default tiling
    recs = sim.step_n(9)
    ref_phi, _, ref_recs, _ = gpu_run(gp, phi0, 16)
    np.testing.assert_array_equal(host(sim.state()[0]), ref_phi)
    assert [r["links_dir"] for r in recs] == [r["links_dir"] for r in ref_recs if r["step"] >= 7]
