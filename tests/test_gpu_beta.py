"""The physical force: Eq. (2) with a^beta dV/dphi, beta = 2 and alpha = 2
(the exact equations; PRS keeps beta = 0, alpha = 3), a(eta) = (eta/eta0)^m.
The force grows as a^beta, so walls thin in comoving units; the runs stay
inside the linearised stability bound the library checks.

Gates as for the PRS force: float32 fields within 1e-5 relative L-inf of the
FP64 oracle after 50 steps, float64 within 1e-12; diagnostics of the same
state bitwise in their counts; multi-step passes bitwise equal to single
steps; the adjoint against the FP64 oracle adjoint (1e-4 float32, 1e-10
float64 relative L2)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1710_10420_amd.inputs import uniform_field
from tests.gpu_util import assert_stats_match, gpu_prs, host, params_pair, rel_linf, say, to_dev, torch_mod

pytestmark = pytest.mark.gpu

PHYS = dict(alpha=2.0, beta=2.0)


def dev(a, f64):
    torch = torch_mod()
    if f64:
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).cuda()
    return to_dev(a)


@pytest.mark.parametrize("shape,deta,steps,f64", [((256, 256), 0.1, 50, False), ((48, 40, 36), 0.1, 30, False),
                                                  ((256, 256), 0.1, 50, True)])
def test_beta_fields_and_records_match_oracle(shape, deta, steps, f64):
    say("beta fields", shape, f64)
    prs = gpu_prs()
    gp, op = params_pair(shape, deta, m=1.0, W0=10.0, diag_every=10, precision=prs.PRS_F64 if f64 else None,
                         **PHYS)
    phi0 = uniform_field(shape, 2).astype(np.float64)
    sim = prs.Sim(gp, phi0=dev(phi0, f64))
    recs = sim.step_n(steps)
    g_phi, g_dphi = (host(t) for t in sim.state())
    o_phi, o_dphi, orecs = O.run(op, phi0.reshape(-1), np.zeros(phi0.size), steps, diag_every=10)
    gate = 1e-12 if f64 else 1e-5
    e = rel_linf(g_phi, o_phi)
    say("  rel L-inf phi %.3g" % e)
    assert e <= gate
    assert rel_linf(g_dphi, o_dphi) <= 10 * gate
    # the record of n = 0 is the oracle's on the seeded field; the final
    # diagnostics are the oracle's on the GPU state
    assert_stats_match(recs[0], orecs[0], ctx="n=0")
    assert_stats_match(sim.wall_stats(), O.stats(op, g_phi, g_dphi, steps), ctx="final")


@pytest.mark.parametrize("shape,tiling", [((264, 200), (2, 16, 1)), ((264, 200), (1, 8, 1)), ((40, 36, 30), (1, 16, 4))])
def test_beta_multi_step_bitwise(shape, tiling):
    """Every pass length gives the single-step fields bit for bit with the
    step-dependent force."""
    say("beta multi-step", shape, tiling)
    prs = gpu_prs()
    deta = 0.1
    gp, _ = params_pair(shape, deta, m=1.0, W0=8.0, diag_every=7, **PHYS)
    phi0 = uniform_field(shape, 5)
    ref = prs.Sim(gp, phi0=to_dev(phi0))
    ref.set_tiling(*tiling)
    ref.set_time_blocking(1)
    r_ref = ref.step_n(41)
    rp = [host(t) for t in ref.state()]
    for T in ((2, 3, 4, 6, 8) if len(shape) == 2 else (2, 3)):
        sim = prs.Sim(gp, phi0=to_dev(phi0))
        sim.set_tiling(*tiling)
        sim.set_time_blocking(T)
        r = sim.step_n(41)
        out = [host(t) for t in sim.state()]
        np.testing.assert_array_equal(out[0], rp[0], err_msg=str(T))
        np.testing.assert_array_equal(out[1], rp[1], err_msg=str(T))
        for a, b in zip(r, r_ref):
            assert_stats_match(a, b, rel=1e-13, ctx=str(T))


@pytest.mark.parametrize("shape,nsteps,K,f64", [((64, 48), 24, 7, False), ((64, 48), 24, 7, True),
                                               ((20, 18, 16), 12, 5, True)])
def test_beta_adjoint_matches_oracle(shape, nsteps, K, f64):
    say("beta adjoint", shape, f64)
    torch = torch_mod()
    prs = gpu_prs()
    deta = 0.1
    gp, op = params_pair(shape, deta, m=1.0, W0=8.0, precision=prs.PRS_F64 if f64 else None, **PHYS)
    phi0 = uniform_field(shape, 9).astype(np.float64)
    sim = prs.Sim(gp, phi0=dev(phi0, f64))
    nb = prs.prs_adjoint_workspace_bytes(gp, nsteps, K)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    gphi = torch.empty_like(sim.phi_a)
    loss, gw = prs.prs_adjoint(sim.ctx, nsteps, K, work.data_ptr(), nb, gphi.data_ptr(), None)
    ref = O.adjoint(op, phi0.reshape(-1), np.zeros(phi0.size), nsteps, ckpt_every=K)
    rel2 = float(np.linalg.norm(host(gphi) - ref["grad_phi"]) / np.linalg.norm(ref["grad_phi"]))
    say("  rel L2 %.3g" % rel2)
    assert rel2 <= (1e-10 if f64 else 1e-4)
    assert loss == pytest.approx(ref["loss"], rel=1e-12 if f64 else 1e-5)
    assert gw == pytest.approx(ref["grad_W0"], rel=1e-9 if f64 else 1e-3)


def test_beta_multi_step_adjoint_bitwise():
    """The adjoint's multi-step passes (forward, recomputation, reverse) with
    the per-step force give the single-step gradient fields bit for bit."""
    say("beta multi-step adjoint")
    torch = torch_mod()
    prs = gpu_prs()
    shape = (200, 130)
    gp, _ = params_pair(shape, 0.1, m=1.0, W0=6.0, **PHYS)
    phi0 = uniform_field(shape, 8)
    out = {}
    for T, scheme in ((1, prs.PRS_ADJ_STORED), (8, prs.PRS_ADJ_STORED), (8, prs.PRS_ADJ_FUSED)):
        sim = prs.Sim(gp, phi0=to_dev(phi0))
        prs.prs_set_adjoint_scheme(sim.ctx, scheme)
        sim.set_tiling(2, 16, 1)
        prs.prs_set_adjoint_tiling(sim.ctx, 2, 16, 1)
        sim.set_time_blocking(T)
        prs.prs_set_adjoint_time_blocking(sim.ctx, T)
        nb = prs.prs_adjoint_workspace_bytes(gp, 40, 16)
        work = torch.empty(nb, dtype=torch.uint8, device="cuda")
        g = torch.empty_like(sim.phi_a)
        loss, gw = prs.prs_adjoint(sim.ctx, 40, 16, work.data_ptr(), nb, g.data_ptr(), None)
        out[(T, scheme)] = (host(g), gw, loss)
    ref = out[(1, prs.PRS_ADJ_STORED)]
    for key, tol in (((8, prs.PRS_ADJ_STORED), 1e-11), ((8, prs.PRS_ADJ_FUSED), 1e-5)):
        np.testing.assert_array_equal(out[key][0], ref[0])
        assert out[key][2] == ref[2]
        assert out[key][1] == pytest.approx(ref[1], rel=tol), key


def test_beta_stability_checked_before_launch():
    """The force grows as a^beta; a call that would reach an unstable step is
    rejected before anything runs, and the state is unchanged."""
    prs = gpu_prs()
    shape = (64, 64)
    gp, _ = params_pair(shape, 0.25, m=1.0, W0=10.0, **PHYS)   # a^2 = 64 at eta ~ 8
    sim = prs.Sim(gp, seed=3)
    before = host(sim.state()[0]).copy()
    with pytest.raises(prs.PRSError) as e:
        sim.step_n(200)
    assert e.value.status == prs.PRS_EINVAL and "unstable" in str(e.value)
    np.testing.assert_array_equal(host(sim.state()[0]), before)
    sim.step_n(10)                                              # eta 1 -> 3.5 is stable


@pytest.mark.parametrize("mode", ["STREAMS", "PERSISTENT", "PERSISTENT_GRAPH", "PER_STEP"])
def test_beta_batch_modes(mode):
    """A physical-force realisation in an ensemble equals the same run alone
    (fields and records bit for bit), in the stream mode and in the
    persistent kernel, whose per-step coefficient table carries the force's
    a^beta factor."""
    say("beta batch", mode)
    prs = gpu_prs()
    specs = [dict(shape=(128, 96), deta=0.1, m=1.0, W0=10.0, nsteps=31, diag_every=5, seed=3),
             dict(shape=(96, 64), deta=0.1, m=1.0, W0=10.0, nsteps=17, diag_every=4, seed=4)]
    b = prs.Batch([dict(sp, alpha=2.0, beta=2.0) if r == 0 else sp for r, sp in enumerate(specs)])
    sims = []
    for r, sp in enumerate(specs):
        extra = PHYS if r == 0 else {}
        p = prs.make_params(sp["shape"], deta=sp["deta"], m=sp["m"], W0=sp["W0"], diag_every=sp["diag_every"],
                            **extra)
        sim = prs.Sim(p, seed=sp["seed"])
        b.set_tiling(r, *sim.tiling())
        b.set_time_blocking(r, sim.time_blocking())
        sims.append(sim)
    b.set_mode(getattr(prs, "PRS_BATCH_" + mode))
    recs = b.run()
    for r, sp in enumerate(specs):
        srecs = sims[r].step_n(sp["nsteps"])
        srecs.append(sims[r].wall_stats())
        phi, _ = b.final_state(r)
        np.testing.assert_array_equal(host(phi), host(sims[r].state()[0]))
        assert recs[r] == srecs
    b.close()
