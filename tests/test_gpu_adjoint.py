"""Parity of the GPU adjoint (prs_adjoint*, PRSLoss) with the FP64 oracle
adjoint.  The GPU differentiates its own float32 trajectory and the oracle
its float64 one, so gradients agree to the trajectory's rounding: relative L2
<= 1e-4 for runs of up to 64 steps (the oracle adjoint itself is pinned to
central finite differences in test_oracle_pins).

dL/dW0 is -2 V0/W0 times dL/dV0 = -sum over steps n and sites i of
b_n w_i phi_i (phi_i^2 - 1): every term carries the float32 trajectory's
relative error (<= 1e-5 in the fields over these lengths, the north-star
field gate) and the sum adds them with mixed signs, so its relative error
is of that order unless the terms cancel; the gate is 1e-5 (the largest
deviation seen over these cases is 1.2e-6)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1710_10420_amd.inputs import uniform_field
from tests.gpu_util import gpu_prs, host, params_pair, say, to_dev, torch_mod

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def gpu_adjoint(gp, phi0, nsteps, K, tiling=None):
    torch = torch_mod()
    prs = gpu_prs()
    sim = prs.Sim(gp, phi0=to_dev(phi0))
    if tiling is not None:
        sim.set_tiling(*tiling)
    nb = prs.prs_adjoint_workspace_bytes(gp, nsteps, K)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    gphi = torch.empty_like(sim.phi_a)
    gdphi = torch.empty_like(sim.phi_a)
    loss, gw = prs.prs_adjoint(sim.ctx, nsteps, K, work.data_ptr(), nb, gphi.data_ptr(),
                               gdphi.data_ptr())
    return loss, host(gphi), host(gdphi), gw, sim


@pytest.mark.parametrize("shape,nsteps,K", [
    ((32, 32), 16, 7), ((32, 32), 48, 16), ((256, 256), 64, 16), ((24, 20, 18), 20, 6),
    ((100, 37), 33, 10), ((37, 20, 11), 12, 64),
])
def test_adjoint_matches_oracle(shape, nsteps, K):
    say("adjoint", shape, nsteps, K)
    deta = 0.25 if len(shape) == 2 else 0.2
    gp, op = params_pair(shape, deta, m=1.0, W0=10.0)
    phi0 = uniform_field(shape, 3)
    loss, gphi, gdphi, gw, _ = gpu_adjoint(gp, phi0, nsteps, K)
    ref = O.adjoint(op, phi0.astype(np.float64).reshape(-1), np.zeros(phi0.size), nsteps,
                    ckpt_every=K)
    say("  rel-L2 %.3g %.3g, dW0 rel %.3g" % (rel_l2(gphi, ref["grad_phi"]), rel_l2(gdphi, ref["grad_pi"]),
                                              abs(gw / ref["grad_W0"] - 1.0)))
    assert loss == pytest.approx(ref["loss"], rel=1e-5)
    assert rel_l2(gphi, ref["grad_phi"]) <= 1e-4
    assert rel_l2(gdphi, ref["grad_pi"]) <= 1e-4
    assert gw == pytest.approx(ref["grad_W0"], rel=1e-5)


def gpu_adjoint_T(gp, phi0, nsteps, K, T, tiling=None, TA=None, rec=None, scheme=None, adj_tiling=None):
    """Adjoint with T steps per forward/recompute pass and TA (default T)
    steps per reverse pass, both on `tiling` (the reverse on `adj_tiling`
    when given); `rec` = (vec, rows, ty, steps) gives the recomputation its
    own setting; `scheme` PRS_ADJ_STORED or PRS_ADJ_FUSED (default: the
    library's)."""
    torch = torch_mod()
    prs = gpu_prs()
    sim = prs.Sim(gp, phi0=to_dev(phi0) if gp.precision == prs.PRS_F32 else
                  torch.from_numpy(np.asarray(phi0, np.float64).reshape(-1)).cuda())
    if scheme is not None:
        prs.prs_set_adjoint_scheme(sim.ctx, scheme)
    if tiling is not None:
        sim.set_tiling(*tiling)
        prs.prs_set_adjoint_tiling(sim.ctx, *tiling)
    if adj_tiling is not None:
        prs.prs_set_adjoint_tiling(sim.ctx, *adj_tiling)
    sim.set_time_blocking(T)
    prs.prs_set_adjoint_time_blocking(sim.ctx, T if TA is None else TA)
    if rec is not None:
        prs.prs_set_recompute_tiling(sim.ctx, *rec)
        assert prs.prs_get_recompute_tiling(sim.ctx) == tuple(rec)
    nb = prs.prs_adjoint_workspace_bytes(gp, nsteps, K)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    gphi = torch.empty_like(sim.phi_a)
    gdphi = torch.empty_like(sim.phi_a)
    loss, gw = prs.prs_adjoint(sim.ctx, nsteps, K, work.data_ptr(), nb, gphi.data_ptr(), gdphi.data_ptr())
    return loss, host(gphi), host(gdphi), gw


def test_adjoint_checkpoint_interval_bitwise():
    """Recomputation is bit-exact, so the gradient does not depend on K
    (single steps: dL/dW0 too, bit for bit)."""
    say("adjoint K invariance")
    shape = (200, 130)
    gp, _ = params_pair(shape, 0.25, m=2.0, W0=5.0)
    phi0 = uniform_field(shape, 4)
    ref = gpu_adjoint_T(gp, phi0, 40, 1, 1)
    for K in (3, 16, 40, 64):
        got = gpu_adjoint_T(gp, phi0, 40, K, 1)
        np.testing.assert_array_equal(got[1], ref[1])
        np.testing.assert_array_equal(got[2], ref[2])
        assert got[3] == ref[3] and got[0] == ref[0]


@pytest.mark.parametrize("shape,nsteps,K,tiling", [
    ((200, 130), 40, 16, (1, 16, 1)), ((264, 200), 37, 10, (2, 17, 1)), ((256, 256), 64, 64, (2, 64, 1)),
    ((130, 9), 23, 7, (2, 8, 1)), ((40, 36, 30), 21, 8, (1, 16, 4)), ((64, 9, 33), 14, 5, (2, 16, 2)),
    ((48, 10, 21), 19, 6, (1, 8, 2)), ((256, 40), 26, 9, (4, 8, 1)),
])
def test_multi_step_adjoint_bitwise_equal_single_steps(shape, nsteps, K, tiling):
    """Multi-step passes in the forward-with-checkpoints, the recomputation
    (storing every step) and the reverse sweep leave the gradient fields bit
    for bit those of single steps, for every steps per pass, checkpoint
    interval and ragged segment; dL/dW0 agrees to summation order."""
    say("multi-step adjoint", shape, nsteps, K, tiling)
    prs = gpu_prs()
    deta = 0.25 if len(shape) == 2 else 0.2
    gp, _ = params_pair(shape, deta, m=1.0, W0=6.0)
    phi0 = uniform_field(shape, 8)
    ref = gpu_adjoint_T(gp, phi0, nsteps, K, 1, tiling, scheme=prs.PRS_ADJ_STORED)
    for scheme in (prs.PRS_ADJ_STORED, prs.PRS_ADJ_FUSED):
        # fused passes sum dL/dV0 per lane in float32 over one group of rows
        # before the double sums, which moves it by a few float32 roundings
        gtol = 1e-11 if scheme == prs.PRS_ADJ_STORED or len(shape) == 3 else 1e-5
        for T in ((2, 3, 4, 6, 8) if len(shape) == 2 else (2, 3)):
            for TA in (1, T, (8 if len(shape) == 2 else 3) if T == 2 else 2):
                got = gpu_adjoint_T(gp, phi0, nsteps, K, T, tiling, TA, scheme=scheme)
                np.testing.assert_array_equal(got[1], ref[1], err_msg=str((scheme, T, TA)))
                np.testing.assert_array_equal(got[2], ref[2], err_msg=str((scheme, T, TA)))
                assert got[0] == ref[0]
                assert got[3] == pytest.approx(ref[3], rel=gtol), (scheme, T, TA, got[3] / ref[3] - 1.0)
    # the recomputation on a tiling and pass length of its own
    rec = (1, 8, 1, 3) if len(shape) == 2 else (1, 8, 4, 3)
    got = gpu_adjoint_T(gp, phi0, nsteps, K, 2, tiling, 2, rec)
    np.testing.assert_array_equal(got[1], ref[1], err_msg=str(rec))
    np.testing.assert_array_equal(got[2], ref[2], err_msg=str(rec))


@pytest.mark.parametrize("shape,nsteps,K", [((200, 130), 41, 16), ((97, 9), 23, 7), ((7, 5), 13, 5),
                                            ((300, 70), 64, 64), ((1, 12), 10, 4)])
@pytest.mark.parametrize("adj_tiling", [(1, 8, 1), (2, 16, 1), (1, 64, 1), (2, 5, 1)])
def test_fused_reverse_passes_bitwise(shape, nsteps, K, adj_tiling):
    """Reverse passes that recompute their fields from pass-start states
    (the fused scheme) leave the gradient fields bit for bit those of single
    reverse steps, for 2, 3 and 4 steps per pass, ragged segments and row
    tiles, lattices narrower and shorter than a tile's halo, and tilings of
    one and two sites per lane; dL/dW0 to float32 partial-sum rounding."""
    say("fused reverse", shape, nsteps, K, adj_tiling)
    prs = gpu_prs()
    if shape[0] % adj_tiling[0]:
        pytest.skip("vec must divide nx")
    gp, _ = params_pair(shape, 0.25, m=1.0, W0=6.0)
    phi0 = uniform_field(shape, 11)
    ref = gpu_adjoint_T(gp, phi0, nsteps, K, 1, scheme=prs.PRS_ADJ_STORED)
    for TA in (2, 3, 4):
        got = gpu_adjoint_T(gp, phi0, nsteps, K, 4, TA=TA, scheme=prs.PRS_ADJ_FUSED, adj_tiling=adj_tiling)
        np.testing.assert_array_equal(got[1], ref[1], err_msg=str(TA))
        np.testing.assert_array_equal(got[2], ref[2], err_msg=str(TA))
        assert got[0] == ref[0]
        assert got[3] == pytest.approx(ref[3], rel=1e-5), (TA, got[3] / ref[3] - 1.0)


def test_fused_reverse_f64():
    """The fused scheme in float64 (one site per lane) against float64
    single reverse steps: gradient fields bit for bit."""
    say("fused reverse f64")
    prs = gpu_prs()
    gp = prs.make_params((130, 96), deta=0.25, m=1.0, W0=6.0, precision=prs.PRS_F64)
    phi0 = uniform_field((130, 96), 9)
    ref = gpu_adjoint_T(gp, phi0, 30, 12, 1, scheme=prs.PRS_ADJ_STORED)
    for TA in (2, 3, 4):
        got = gpu_adjoint_T(gp, phi0, 30, 12, 4, TA=TA, scheme=prs.PRS_ADJ_FUSED, adj_tiling=(1, 16, 1))
        np.testing.assert_array_equal(got[1], ref[1], err_msg=str(TA))
        np.testing.assert_array_equal(got[2], ref[2], err_msg=str(TA))
        assert got[3] == pytest.approx(ref[3], rel=1e-12), TA


@pytest.mark.parametrize("shape,tiling", [((130, 96), (2, 16, 1)), ((130, 96), (1, 8, 1)),
                                          ((40, 36, 30), (1, 16, 2))])
def test_multi_step_adjoint_f64(shape, tiling):
    say("multi-step adjoint f64", shape)
    prs = gpu_prs()
    deta = 0.25 if len(shape) == 2 else 0.2
    gp = prs.make_params(shape, deta=deta, m=1.0, W0=6.0, precision=prs.PRS_F64)
    phi0 = uniform_field(shape, 9)
    ref = gpu_adjoint_T(gp, phi0, 30, 12, 1, tiling)
    for T in ((2, 3, 4, 6, 8) if len(shape) == 2 else (2,)):
        got = gpu_adjoint_T(gp, phi0, 30, 12, T, tiling)
        np.testing.assert_array_equal(got[1], ref[1], err_msg=str(T))
        np.testing.assert_array_equal(got[2], ref[2], err_msg=str(T))
        assert got[3] == pytest.approx(ref[3], rel=1e-13), T


def test_adjoint_backward_requires_forward():
    prs = gpu_prs()
    torch = torch_mod()
    shape = (64, 64)
    gp, _ = params_pair(shape, 0.25)
    sim = prs.Sim(gp, seed=1)
    nb = prs.prs_adjoint_workspace_bytes(gp, 8, 4)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    with pytest.raises(prs.PRSError) as e:
        prs.prs_adjoint_backward(sim.ctx, work.data_ptr(), nb, None, None)
    assert e.value.status == prs.PRS_ESTATE
    with pytest.raises(prs.PRSError) as e:
        prs.prs_adjoint_forward(sim.ctx, 8, 4, work.data_ptr(), nb - 256)
    assert e.value.status == prs.PRS_ENOMEM


def test_prsloss_autograd():
    """PRSLoss routes loss.backward() through the hand-written adjoint."""
    say("PRSLoss autograd")
    torch = torch_mod()
    prs = gpu_prs()
    shape = (128, 96)
    gp, op = params_pair(shape, 0.25, m=1.0, W0=8.0)
    phi0_np = uniform_field(shape, 12)
    phi0 = to_dev(phi0_np).requires_grad_(True)
    W0 = torch.tensor(8.0, dtype=torch.float64, requires_grad=True)
    loss = prs.PRSLoss.apply(phi0, W0, gp, 30, 8)
    (2.0 * loss).backward()
    ref = O.adjoint(op, phi0_np.astype(np.float64).reshape(-1), np.zeros(phi0_np.size), 30,
                    ckpt_every=8)
    assert float(loss) == pytest.approx(ref["loss"], rel=1e-5)
    assert rel_l2(host(phi0.grad) / 2.0, ref["grad_phi"]) <= 1e-4
    assert float(W0.grad) / 2.0 == pytest.approx(ref["grad_W0"], rel=1e-5)


@pytest.mark.parametrize("shape,nsteps,K,tuned", [
    ((2048, 2048), 64, 64, ((2, 16, 1), 8, (1, 32, 1), 8)),
    ((256, 256, 256), 16, 8, ((1, 16, 4), 3, (1, 16, 2), 3)),
])
def test_adjoint_full_size(shape, nsteps, K, tuned):
    """The adjoint at the full lattice sizes (2048^2, 256^3), over runs the
    oracle finishes in seconds, with the library defaults and with the
    configuration the benchmark's tuners pick (forward and recomputation
    tiling and steps per pass, reverse tiling and steps per pass)."""
    say("adjoint full size", shape)
    torch = torch_mod()
    prs = gpu_prs()
    deta = 0.25 if len(shape) == 2 else 0.2
    gp, op = params_pair(shape, deta, m=1.0, W0=10.0)
    phi0 = uniform_field(shape, 7)
    O.set_threads(16)
    ref = O.adjoint(op, phi0.astype(np.float64).reshape(-1), np.zeros(phi0.size), nsteps,
                    ckpt_every=K)
    for cfg in (None, tuned):
        sim = prs.Sim(gp, phi0=to_dev(phi0))
        if cfg is not None:
            sim.set_tiling(*cfg[0])
            sim.set_time_blocking(cfg[1])
            prs.prs_set_adjoint_tiling(sim.ctx, *cfg[2])
            prs.prs_set_adjoint_time_blocking(sim.ctx, cfg[3])
        say("  tiling", sim.tiling(), "steps/pass", sim.time_blocking())
        nb = prs.prs_adjoint_workspace_bytes(gp, nsteps, K)
        work = torch.empty(nb, dtype=torch.uint8, device="cuda")
        gphi = torch.empty_like(sim.phi_a)
        gdphi = torch.empty_like(sim.phi_a)
        loss, gw = prs.prs_adjoint(sim.ctx, nsteps, K, work.data_ptr(), nb, gphi.data_ptr(), gdphi.data_ptr())
        say("  rel-L2 %.3g, dW0 rel %.3g" % (rel_l2(host(gphi), ref["grad_phi"]), abs(gw / ref["grad_W0"] - 1.0)))
        assert loss == pytest.approx(ref["loss"], rel=1e-5), cfg
        assert rel_l2(host(gphi), ref["grad_phi"]) <= 1e-4, cfg
        assert rel_l2(host(gdphi), ref["grad_pi"]) <= 1e-4, cfg
        assert gw == pytest.approx(ref["grad_W0"], rel=1e-5), cfg
        del sim, work, gphi, gdphi
        torch.cuda.empty_cache()


@pytest.mark.parametrize("shape", [(200, 130), (40, 36, 30)])
def test_adjoint_tiling_independent(shape):
    """The reverse-sweep kernel's tiling changes nothing but the summation
    order of dL/dW0: gradient fields are bitwise equal."""
    say("adjoint tilings", shape)
    torch = torch_mod()
    prs = gpu_prs()
    deta = 0.25 if len(shape) == 2 else 0.2
    gp, _ = params_pair(shape, deta, m=1.0, W0=8.0)
    phi0 = uniform_field(shape, 5)
    nb = prs.prs_adjoint_workspace_bytes(gp, 20, 8)
    ref = None
    for scheme in (prs.PRS_ADJ_STORED, prs.PRS_ADJ_FUSED):
        # the fused scheme's float32 partial sums move dL/dW0 by a few roundings
        gtol = 1e-12 if scheme == prs.PRS_ADJ_STORED or len(shape) == 3 else 1e-5
        for t in [(1, 8, 1), (2, 17, 1), (4, 64, 1)] + ([(2, 16, 2), (1, 32, 4)] if len(shape) == 3 else []):
            if shape[0] % t[0]:
                continue
            sim = prs.Sim(gp, phi0=to_dev(phi0))
            prs.prs_set_adjoint_scheme(sim.ctx, scheme)
            prs.prs_set_adjoint_tiling(sim.ctx, *t)
            work = torch.empty(nb, dtype=torch.uint8, device="cuda")
            g = torch.empty_like(sim.phi_a)
            loss, gw = prs.prs_adjoint(sim.ctx, 20, 8, work.data_ptr(), nb, g.data_ptr(), None)
            if ref is None:
                ref = (host(g), gw, loss)
                continue
            np.testing.assert_array_equal(host(g), ref[0])
            assert gw == pytest.approx(ref[1], rel=gtol) and loss == ref[2], (scheme, t)


@pytest.mark.parametrize("shape", [(256, 192), (64, 40, 36)])
def test_adjoint_autotune_picks_reverse_passes(shape):
    """PRS_TUNE_ADJOINT chooses the reverse tiling and steps per pass
    together; the gradient is unchanged by the choice."""
    say("adjoint tuner", shape)
    prs = gpu_prs()
    torch = torch_mod()
    deta = 0.25 if len(shape) == 2 else 0.2
    gp, _ = params_pair(shape, deta, m=1.0, W0=8.0)
    phi0 = uniform_field(shape, 6)
    ref = gpu_adjoint_T(gp, phi0, 24, 8, 1, (2, 16, 1), 1)
    sim = prs.Sim(gp, phi0=to_dev(phi0))
    sim.set_tiling(2, 16, 1)
    sim.set_time_blocking(1)
    prs.prs_autotune(sim.ctx, None, prs.PRS_TUNE_ADJOINT | prs.PRS_TUNE_FORCE)
    TA = prs.prs_get_adjoint_time_blocking(sim.ctx)
    assert TA in (1, 2, 3, 4, 8)
    nb = prs.prs_adjoint_workspace_bytes(gp, 24, 8)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    g = torch.empty_like(sim.phi_a)
    loss, gw = prs.prs_adjoint(sim.ctx, 24, 8, work.data_ptr(), nb, g.data_ptr(), None)
    np.testing.assert_array_equal(host(g), ref[1])
    fused = len(shape) == 2 and prs.prs_get_adjoint_scheme(sim.ctx) == prs.PRS_ADJ_FUSED
    assert gw == pytest.approx(ref[3], rel=1e-5 if fused else 1e-11)


def cosine(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-300))


@pytest.mark.slow
@pytest.mark.timeout(1500)
@pytest.mark.parametrize("shape", [(2048, 2048), (256, 256, 256)])
def test_adjoint_full_length(shape):
    """The adjoint workload at its stated length: 1024 steps from seed 7
    (m = 1, W0 = 10), checkpoints every 64 steps, so 16 segments and the
    recomputation of every older segment overlapping the sweep of the newer
    one; forward and reverse settings from the library's tuners, as the
    benchmark runs it.  The float32 trajectory drifts from the float64 one
    over 1024 chaotic steps, so the gates are on direction and size rather
    than elementwise: cosine similarity >= 0.999 for dL/dphi0 and
    dL/dphi_dot0, |dW0 - dW0_ref| <= 1e-2 |dW0_ref|, loss to 1e-3.  The
    relative L2 distance is printed."""
    torch = torch_mod()
    prs = gpu_prs()
    nsteps, K = 1024, 64
    deta = 0.25 if len(shape) == 2 else 0.2
    gp, op = params_pair(shape, deta, m=1.0, W0=10.0)
    phi0 = uniform_field(shape, 7)
    say("adjoint full length", shape, "oracle ...")
    O.set_threads(min(16, len(__import__("os").sched_getaffinity(0))))
    O.set_progress(True)
    try:
        ref = O.adjoint(op, phi0.astype(np.float64).reshape(-1), np.zeros(phi0.size), nsteps,
                        ckpt_every=K)
    finally:
        O.set_progress(False)
    say("  oracle done; GPU ...")
    sim = prs.Sim(gp, phi0=to_dev(phi0))
    prs.prs_autotune(sim.ctx, None, 0)
    prs.prs_autotune(sim.ctx, None, prs.PRS_TUNE_ADJOINT)
    say("  tiling", sim.tiling(), "steps/pass", sim.time_blocking(), "reverse",
        prs.prs_get_adjoint_tiling(sim.ctx), prs.prs_get_adjoint_time_blocking(sim.ctx))
    nb = prs.prs_adjoint_workspace_bytes(gp, nsteps, K)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    gphi = torch.empty_like(sim.phi_a)
    gdphi = torch.empty_like(sim.phi_a)
    loss, gw = prs.prs_adjoint(sim.ctx, nsteps, K, work.data_ptr(), nb, gphi.data_ptr(), gdphi.data_ptr())
    g, gd = host(gphi), host(gdphi)
    c_phi, c_pi = cosine(g, ref["grad_phi"]), cosine(gd, ref["grad_pi"])
    say("  loss %.9g / %.9g, cos(dphi0) %.7f rel-L2 %.3g, cos(dpi0) %.7f rel-L2 %.3g, dW0 %.7g / %.7g"
        % (loss, ref["loss"], c_phi, rel_l2(g, ref["grad_phi"]), c_pi, rel_l2(gd, ref["grad_pi"]),
           gw, ref["grad_W0"]))
    assert loss == pytest.approx(ref["loss"], rel=1e-3)
    assert c_phi >= 0.999 and c_pi >= 0.999
    assert abs(gw - ref["grad_W0"]) <= 1e-2 * abs(ref["grad_W0"])
    sim.close()
    del sim, work, gphi, gdphi
    torch.cuda.empty_cache()
