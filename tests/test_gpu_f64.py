"""The float64 instantiation of the kernels (PRS_F64; the paper runs its
kernels in both precisions, Sec. III and Table I).

Gates.  The float64 GPU path and the FP64 oracle evaluate Eqs. (3)-(6) with
different operation orders (the GPU forms the kick with fused multiply-adds
and precomputed a_n, b_n; the oracle divides by 1 + delta), so their fields
differ by a few units of roundoff per step, carried along by the dynamics.
The float32 gate is 1e-5 relative L-inf after 50 steps of the 256^2 case;
scaling it by the ratio of unit roundoffs (2^-53 / 2^-24 ~ 1.9e-9) gives
~2e-14, and the gate here is 1e-12 (the float32 path's observed error is
~40x below its gate, so this leaves a similar margin for the different
fused-multiply-add placement).  Counts are bitwise on the same field; the
adjoint agrees with the oracle adjoint to 1e-10 relative L2; and
torch.autograd.gradcheck checks the float64 adjoint against central finite
differences of the float64 GPU forward itself."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1710_10420_amd.inputs import uniform_field
from tests.gpu_util import assert_stats_match, gpu_prs, host, rel_linf, say, torch_mod

pytestmark = pytest.mark.gpu

F64_FIELD_GATE = 1e-12


def params64(shape, deta, **kw):
    prs = gpu_prs()
    gp = prs.make_params(shape, deta=deta, precision=prs.PRS_F64, **kw)
    okw = {k: v for k, v in kw.items() if k != "diag_every"}
    op = O.params(shape, deta=deta, **okw)
    return gp, op


def dev64(a):
    torch = torch_mod()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).cuda()


def test_fill_uniform_f64_is_the_float32_field():
    say("fill f64")
    torch = torch_mod()
    prs = gpu_prs()
    n = 300 * 77
    s = prs._stream_handle(torch.cuda.current_stream())
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.empty(n, dtype=torch.float32, device="cuda")
    prs.prs_fill_uniform_f64(a.data_ptr(), n, 11, s)
    prs.prs_fill_uniform(b.data_ptr(), n, 11, s)
    np.testing.assert_array_equal(host(a), host(b).astype(np.float64))
    np.testing.assert_array_equal(host(a), uniform_field((300, 77), 11).reshape(-1).astype(np.float64))


@pytest.mark.parametrize("shape,deta,steps", [((256, 256), 0.25, 50), ((48, 40, 36), 0.2, 30)])
def test_f64_fields_match_oracle(shape, deta, steps):
    say("f64 fields", shape, steps)
    prs = gpu_prs()
    gp, op = params64(shape, deta, m=1.0, W0=10.0, diag_every=10)
    phi0 = uniform_field(shape, 1).astype(np.float64)
    sim = prs.Sim(gp, phi0=dev64(phi0))
    assert sim.phi_a.dtype == torch_mod().float64
    sim.step_n(steps)
    g_phi, g_dphi = (host(t) for t in sim.state())
    o_phi, o_dphi, _ = O.run(op, phi0, np.zeros(phi0.size), steps)
    e_phi, e_dphi = rel_linf(g_phi, o_phi), rel_linf(g_dphi, o_dphi)
    say("  rel L-inf phi %.3g dphi %.3g" % (e_phi, e_dphi))
    assert e_phi <= F64_FIELD_GATE
    assert e_dphi <= 10 * F64_FIELD_GATE
    st = sim.wall_stats()
    assert_stats_match(st, O.stats(op, g_phi, g_dphi, steps), ctx="f64 %s" % (shape,))


def test_f64_fused_records_and_full_run():
    """Every fused record of a full 256^2 run (508 steps, records every 10)
    equals the oracle diagnostics of the GPU state it was taken on (counts
    bitwise), and the run's fitted exponents agree with the oracle run's."""
    say("f64 full run")
    prs = gpu_prs()
    shape = (256, 256)
    gp, op = params64(shape, 0.25, m=1.0, W0=10.0, diag_every=10)
    phi0 = uniform_field(shape, 2).astype(np.float64)
    sim = prs.Sim(gp, phi0=dev64(phi0))
    grecs = []
    for n in range(0, 508, 100):
        phi, dphi = sim.state()
        o = O.stats(op, host(phi), host(dphi), n)
        recs = sim.step_n(min(100, 508 - n))
        assert_stats_match(recs[0], o, rel=1e-12, ctx="n=%d" % n)
        grecs += recs
    grecs.append(sim.wall_stats())
    o_phi, o_dphi, orecs = O.run(op, phi0, np.zeros(phi0.size), 508, diag_every=10)
    orecs.append(O.stats(op, o_phi, o_dphi, 508))
    gmu, gnu = prs.prs_fit_scaling(grecs, 12.8)
    omu, onu = O.scaling_exponents(orecs, 12.8)
    say("  mu gpu %.6f oracle %.6f" % (gmu, omu))
    assert abs(gmu - omu) <= 0.02 and abs(gnu - onu) <= 0.05


@pytest.mark.parametrize("shape", [(264, 200), (40, 36, 30)])
def test_f64_tiling_and_steps_per_pass_independence(shape):
    """Fields are bitwise independent of the tiling (vec 1, 2; 3D rows of
    1, 2, 4) and of the steps per pass (2D: 1 .. 8, the six- and eight-step
    passes with vec 1 and, asked of vec 2, the planner's shorter passes; 3D:
    1, 2)."""
    say("f64 tilings", shape)
    prs = gpu_prs()
    deta = 0.25 if len(shape) == 2 else 0.2
    gp, _ = params64(shape, deta, m=2.0, W0=6.0, diag_every=7)
    phi0 = dev64(uniform_field(shape, 5))
    ref = None
    tys = (1,) if len(shape) == 2 else (1, 2, 4)
    for vec in (1, 2):
        for rows in (8, 17):
            for ty in tys:
                for T in ((1, 2, 3, 4, 6, 8) if len(shape) == 2 else (1, 2)):
                    sim = prs.Sim(gp, phi0=phi0)
                    sim.set_tiling(vec, rows, ty)
                    sim.set_time_blocking(T)
                    recs = sim.step_n(23)
                    out = [host(t) for t in sim.state()]
                    if ref is None:
                        ref = (out, recs)
                        continue
                    np.testing.assert_array_equal(out[0], ref[0][0], err_msg=str((vec, rows, ty, T)))
                    np.testing.assert_array_equal(out[1], ref[0][1], err_msg=str((vec, rows, ty, T)))
                    for a, b in zip(recs, ref[1]):
                        assert_stats_match(a, b, rel=1e-13, ctx=str((vec, rows, ty, T)))


def test_f64_full_size_sampled():
    """8192^2 matter era in float64 in the configuration the float64
    benchmark leg's tuner picks (one site per lane, 128 rows, eight steps per
    pass): sampled patches after 64 steps match the FP64 oracle evolved on
    each patch's dependence cone to the float64 gate."""
    say("f64 8192^2 full size")
    torch = torch_mod()
    prs = gpu_prs()
    from tests.gpu_util import oracle_patch
    shape = (8192, 8192)
    gp, op = params64(shape, 0.25, m=2.0, W0=10.0, diag_every=64)
    sim = prs.Sim(gp, seed=1)
    sim.set_tiling(1, 128, 1)
    sim.set_time_blocking(8)
    assert prs.prs_plan_passes(sim.ctx, 64)[0] >= 1
    sim.step_n(64)
    g = host(sim.state()[0])
    rng = np.random.default_rng(8)
    centers = [(0, 0), (8191, 8191), (4095, 17)] + [tuple(int(v) for v in rng.integers(0, 8192, 2))
                                                    for _ in range(3)]
    for c in centers:
        idx, ref = oracle_patch(op, shape, 1, c, 64, 6)
        assert rel_linf(g[idx], ref) <= F64_FIELD_GATE, c
    del sim
    torch.cuda.empty_cache()


def test_f64_rejects_four_sites_per_lane():
    prs = gpu_prs()
    gp, _ = params64((256, 64), 0.25)
    sim = prs.Sim(gp, seed=1)
    assert sim.tiling()[0] in (1, 2)
    with pytest.raises(prs.PRSError) as e:
        sim.set_tiling(4, 16, 1)
    assert e.value.status == prs.PRS_EINVAL


@pytest.mark.parametrize("shape,nsteps,K", [((64, 48), 24, 7), ((20, 18, 16), 12, 5)])
def test_f64_adjoint_matches_oracle(shape, nsteps, K):
    say("f64 adjoint", shape)
    torch = torch_mod()
    prs = gpu_prs()
    deta = 0.25 if len(shape) == 2 else 0.2
    gp, op = params64(shape, deta, m=1.0, W0=8.0)
    phi0 = uniform_field(shape, 9).astype(np.float64)
    sim = prs.Sim(gp, phi0=dev64(phi0))
    nb = prs.prs_adjoint_workspace_bytes(gp, nsteps, K)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    gphi = torch.empty_like(sim.phi_a)
    gdphi = torch.empty_like(sim.phi_a)
    loss, gw = prs.prs_adjoint(sim.ctx, nsteps, K, work.data_ptr(), nb, gphi.data_ptr(), gdphi.data_ptr())
    ref = O.adjoint(op, phi0.reshape(-1), np.zeros(phi0.size), nsteps, ckpt_every=K)
    rel2 = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    assert loss == pytest.approx(ref["loss"], rel=1e-12)
    assert rel2(host(gphi), ref["grad_phi"]) <= 1e-10
    assert rel2(host(gdphi), ref["grad_pi"]) <= 1e-10
    assert gw == pytest.approx(ref["grad_W0"], rel=1e-9)


def test_f64_gradcheck():
    """torch.autograd.gradcheck of PRSLoss in float64 on the GPU: the
    hand-written reverse sweep against central differences of the forward
    evolution, for phi0 and W0."""
    say("f64 gradcheck")
    torch = torch_mod()
    prs = gpu_prs()
    shape = (12, 10)
    gp = prs.make_params(shape, deta=0.25, m=1.0, W0=3.0)
    phi0 = torch.from_numpy(uniform_field(shape, 4).reshape(-1).astype(np.float64)).cuda()
    phi0.requires_grad_(True)
    W0 = torch.tensor(3.0, dtype=torch.float64, requires_grad=True)
    f = lambda a, w: prs.PRSLoss.apply(a, w, gp, 10, 4)
    assert torch.autograd.gradcheck(f, (phi0, W0), eps=1e-6, atol=1e-7, rtol=1e-5)


def test_f64_batch_stream_mode():
    """float64 realisations in a batch (stream modes) equal the same runs
    alone; the persistent modes refuse them."""
    say("f64 batch")
    prs = gpu_prs()
    specs = [dict(shape=(128, 96), deta=0.25, m=1.0, W0=10.0, nsteps=21, diag_every=5, seed=3,
                  precision=prs.PRS_F64),
             dict(shape=(24, 20, 18), deta=0.2, m=0.5, W0=5.0, nsteps=9, diag_every=4, seed=4,
                  precision=prs.PRS_F64),
             dict(shape=(64, 64), deta=0.25, m=2.0, W0=10.0, nsteps=13, diag_every=6, seed=5)]
    b = prs.Batch(specs)
    sims = []
    for r, sp in enumerate(specs):
        p = prs.make_params(sp["shape"], deta=sp["deta"], m=sp["m"], W0=sp["W0"],
                            diag_every=sp["diag_every"], precision=sp.get("precision", prs.PRS_F32))
        sim = prs.Sim(p, seed=sp["seed"])
        b.set_tiling(r, *sim.tiling())
        b.set_time_blocking(r, sim.time_blocking())
        sims.append(sim)
    b.set_mode(prs.PRS_BATCH_STREAMS)
    recs = b.run()
    for r, sp in enumerate(specs):
        sim = sims[r]
        srecs = sim.step_n(sp["nsteps"])
        srecs.append(sim.wall_stats())
        phi, dphi = b.final_state(r)
        np.testing.assert_array_equal(host(phi), host(sim.state()[0]))
        np.testing.assert_array_equal(host(dphi), host(sim.state()[1]))
        assert recs[r] == srecs
    b.set_mode(prs.PRS_BATCH_PERSISTENT)
    with pytest.raises(prs.PRSError) as e:
        b.run()
    assert e.value.status == prs.PRS_EINVAL
    b.close()
