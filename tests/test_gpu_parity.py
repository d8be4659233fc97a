"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Tolerances: the FP32 field must stay within 1e-5 relative L-inf
(max|phi_gpu - phi_ref| / max|phi_ref|) of the FP64 oracle started from the
same field; crossing-link, wall-site and non-finite counts must match bit for
bit when both sides see the same field; the two FP64 diagnostic sums may
differ only by summation order (1e-12 relative).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1710_10420_amd.inputs import uniform_field
from tests import fields as F
from tests.gpu_util import (assert_stats_match, gpu_prs, gpu_run, host, oracle_patch, params_pair,
                            rel_linf, say, to_dev, torch_mod)

pytestmark = pytest.mark.gpu


def oracle_stats_of(op, phi, dphi, n):
    return O.stats(op, np.asarray(phi, np.float64), np.asarray(dphi, np.float64), n)


# ------------------------------------------------------------ generator ----

@pytest.mark.parametrize("count,seed", [(1, 3), (1000, 7), (256 * 256, 1), (8192 * 8192, 1)])
def test_fill_uniform_bitwise(count, seed):
    say("fill_uniform", count, seed)
    torch = torch_mod()
    prs = gpu_prs()
    t = torch.empty(count, dtype=torch.float32, device="cuda")
    prs.prs_fill_uniform(t.data_ptr(), count, seed, prs._stream_handle(torch.cuda.current_stream()))
    got = host(t)
    want = uniform_field((count, 1), seed).reshape(-1)
    np.testing.assert_array_equal(got, want)


# ------------------------------------------------------------ C1 parity ----

@pytest.mark.parametrize("seed", [1, 2])
def test_c1_fields_within_1e5_after_50_steps(seed):
    """North-star gate: 256^2 radiation era, deta 0.25, 50 steps."""
    say("c1 fields", seed)
    shape = (256, 256)
    gp, op = params_pair(shape, 0.25, m=1.0, W0=10.0, diag_every=10)
    phi0 = uniform_field(shape, seed)
    g_phi, g_dphi, recs, sim = gpu_run(gp, phi0, 50)
    o_phi, o_dphi, _ = O.run(op, phi0.astype(np.float64), np.zeros(phi0.size), 50)
    assert rel_linf(g_phi, o_phi) <= 1e-5
    assert rel_linf(g_dphi, o_dphi) <= 1e-4
    assert [r["step"] for r in recs] == [0, 10, 20, 30, 40]
    # standalone diagnostics of the GPU state equal the oracle's on that field
    st = sim.wall_stats()
    assert_stats_match(st, oracle_stats_of(op, g_phi, g_dphi, 50), ctx="c1 n=50")


@pytest.mark.parametrize("T", [1, 2, 4])
def test_c1_fused_records_match_oracle_on_same_field(T):
    """Every fused record equals the oracle diagnostics of the GPU state it
    was taken on (counts bitwise) and the standalone diagnostics of that
    state: bit for bit from single-step passes, up to summation order from
    multi-step passes (different wave tiles)."""
    say("c1 fused records", T)
    shape = (256, 256)
    gp, op = params_pair(shape, 0.25, m=1.0, W0=10.0, diag_every=10)
    prs = gpu_prs()
    sim = prs.Sim(gp, phi0=to_dev(uniform_field(shape, 3)))
    sim.set_time_blocking(T)
    for n in range(0, 60, 10):
        phi, dphi = sim.state()
        standalone = sim.wall_stats()
        o = oracle_stats_of(op, host(phi), host(dphi), n)
        assert_stats_match(standalone, o, ctx="n=%d" % n)
        recs = sim.step_n(10)
        assert len(recs) == 1
        if T == 1:
            assert recs[0] == standalone      # fused == standalone, bit for bit
        else:
            assert_stats_match(recs[0], standalone, rel=1e-13, ctx="fused n=%d" % n)


def test_c1_full_run_scaling_exponent():
    """Full 256^2 run (eta 1 -> 128, 508 steps): the fitted wall-area
    exponent agrees with the oracle's within 0.02 (the dynamics is chaotic,
    so only fitted exponents are compared over full runs)."""
    shape = (256, 256)
    gp, op = params_pair(shape, 0.25, m=1.0, W0=10.0, diag_every=10)
    prs = gpu_prs()
    for seed in (1, 2, 3, 4, 5):
        say("c1 full run", seed)
        phi0 = uniform_field(shape, seed)
        _, _, grecs, sim = gpu_run(gp, phi0, 508)
        grecs.append(sim.wall_stats())
        o_phi, o_dphi, orecs = O.run(op, phi0.astype(np.float64), np.zeros(phi0.size), 508,
                                     diag_every=10)
        orecs.append(O.stats(op, o_phi, o_dphi, 508))
        eta_min = 12.8   # last decade of eta 1 -> 128
        gmu, gnu = prs.prs_fit_scaling(grecs, eta_min)
        omu, onu = O.scaling_exponents(orecs, eta_min)
        assert abs(gmu - omu) <= 0.02, (seed, gmu, omu)
        assert abs(gnu - onu) <= 0.05, (seed, gnu, onu)


def c2_golden():
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_oracle_records.json")
    with open(path) as f:
        return json.load(f)


@pytest.mark.slow
@pytest.mark.parametrize("tuned", [True, False])
def test_c2_full_run_scaling_exponent(tuned):
    """The 2D matter-era run at full size and length (8192^2, W0 = 10, m = 2,
    deta = 0.25, eta 1 -> 4096, seed 1, records every 64 steps and of the
    final state) against the FP64 oracle's run of the same input, stored in
    tests/golden/c2_oracle_records.json by tests/golden/make_c2_records.py:
    the wall-area exponent fitted over the last decade within 0.02; the
    record of n = 0 (both sides on the same seeded field) with counts bit for
    bit and FP64 sums to summation order; with the benchmark's tuned launch
    configuration and with the library default."""
    gold = c2_golden()
    run = gold["run"]
    prs = gpu_prs()
    shape = tuple(run["shape"])
    gp = prs.make_params(shape, deta=run["deta"], m=run["m"], W0=run["W0"], alpha=run["alpha"],
                         diag_every=run["diag_every"])
    sim = prs.Sim(gp, seed=run["seed"])
    if tuned:
        prs.prs_autotune(sim.ctx, None, 0)
    say("c2 full run", sim.tiling(), sim.time_blocking())
    recs = sim.step_n(gold["steps"])
    recs.append(sim.wall_stats())
    orecs = gold["records"]
    assert len(recs) == len(orecs) == 257
    assert [r["step"] for r in recs] == [r["step"] for r in orecs]
    assert_stats_match(recs[0], orecs[0], ctx="c2 n=0")
    mu, nu = prs.prs_fit_scaling(recs, gold["fit_eta_min"])
    say("  mu %.5f (oracle %.5f), nu %.5f (oracle %.5f)" % (mu, gold["mu"], nu, gold["nu"]))
    assert abs(mu - gold["mu"]) <= 0.02
    assert abs(nu - gold["nu"]) <= 0.05
    sim.close()


# ---------------------------------------------------- ragged / degenerate --

SHAPES = [
    (300, 70), (100, 37), (1, 1), (1, 7), (7, 1), (2, 2), (66, 129), (1030, 9),
    (37, 20, 11), (64, 3, 5), (130, 9, 7), (1, 1, 1), (2, 3, 4), (5, 1, 3), (260, 6, 4),
]


@pytest.mark.parametrize("shape", SHAPES)
def test_ragged_shapes(shape):
    say("ragged", shape)
    deta = 0.25 if len(shape) == 2 else 0.2
    gp, op = params_pair(shape, deta, m=2.0, W0=5.0, diag_every=4)
    phi0 = uniform_field(shape, 17)
    steps = 12
    g_phi, g_dphi, recs, sim = gpu_run(gp, phi0, steps)
    o_phi, o_dphi, _ = O.run(op, phi0.astype(np.float64), np.zeros(phi0.size), steps)
    assert rel_linf(g_phi, o_phi) <= 1e-5
    assert len(recs) == 3
    assert_stats_match(sim.wall_stats(), oracle_stats_of(op, g_phi, g_dphi, steps), ctx=str(shape))


# ------------------------------------------------------------ invariances --

def tilings_for(shape):
    prs = gpu_prs()
    out = []
    nx = shape[0]
    for vec in (1, 2, 4):
        if nx % vec:
            continue
        for rows in (16, 17, 64):
            for ty in ((1,) if len(shape) == 2 else (1, 2, 4)):
                out.append((vec, rows, ty))
    return out


@pytest.mark.parametrize("shape", [(264, 200), (136, 24, 40)])
def test_tiling_independence(shape):
    """Fields and counts are bitwise identical for every tiling; FP64 sums
    differ only by summation order."""
    say("tilings", shape)
    deta = 0.25 if len(shape) == 2 else 0.2
    gp, _ = params_pair(shape, deta, m=1.0, W0=8.0, diag_every=5)
    phi0 = uniform_field(shape, 21)
    ref = None
    for t in tilings_for(shape):
        say("  tiling", t)
        phi, dphi, recs, _ = gpu_run(gp, phi0, 11, tiling=t)
        if ref is None:
            ref = (phi, dphi, recs)
            continue
        np.testing.assert_array_equal(phi, ref[0])
        np.testing.assert_array_equal(dphi, ref[1])
        for a, b in zip(recs, ref[2]):
            assert_stats_match(a, b, rel=1e-13, ctx=str(t))


@pytest.mark.parametrize("shape,shift", [((300, 70), (67, 13)), ((130, 9, 7), (65, 4, 3))])
def test_translation_bitwise(shape, shift):
    """A periodic shift by non-tile multiples commutes with the GPU step."""
    say("translation", shape)
    deta = 0.25 if len(shape) == 2 else 0.2
    gp, _ = params_pair(shape, deta, m=1.0, W0=6.0, diag_every=4)
    phi0 = uniform_field(shape, 5)
    axes = tuple(range(len(shape) - 1, -1, -1))
    roll = lambda a: np.roll(a.reshape(phi0.shape), shift, axis=axes).reshape(-1)
    a, pa, ra, _ = gpu_run(gp, phi0, 9)
    b, pb, rb, _ = gpu_run(gp, roll(phi0), 9)
    np.testing.assert_array_equal(roll(a), b)
    np.testing.assert_array_equal(roll(pa), pb)
    for x, y in zip(ra, rb):
        assert x["links_dir"] == y["links_dir"] and x["wall_sites"] == y["wall_sites"]


@pytest.mark.parametrize("shape", [(256, 256), (40, 30, 20)])
def test_z2_and_vacuum_bitwise(shape):
    say("z2/vacuum", shape)
    deta = 0.25 if len(shape) == 2 else 0.2
    gp, _ = params_pair(shape, deta, m=2.0, W0=10.0, diag_every=5)
    phi0 = uniform_field(shape, 9)
    a, pa, ra, _ = gpu_run(gp, phi0, 15)
    b, pb, rb, _ = gpu_run(gp, -phi0, 15)
    np.testing.assert_array_equal(a, -b)
    np.testing.assert_array_equal(pa, -pb)
    assert [r["links_dir"] for r in ra] == [r["links_dir"] for r in rb]
    for sign in (1.0, -1.0):
        v = np.full(phi0.size, sign, dtype=np.float32)
        c, pc, rc, _ = gpu_run(gp, v, 15)
        np.testing.assert_array_equal(c, v)
        assert np.all(pc == 0.0)
        assert all(r["links"] == 0 and r["wall_sites"] == 0 for r in rc)


def test_split_calls_and_determinism():
    say("split/determinism")
    shape = (512, 300)
    gp, _ = params_pair(shape, 0.25, m=1.0, W0=10.0, diag_every=8)
    phi0 = uniform_field(shape, 4)
    prs = gpu_prs()
    a, pa, ra, _ = gpu_run(gp, phi0, 37)
    a2, pa2, ra2, _ = gpu_run(gp, phi0, 37)
    np.testing.assert_array_equal(a, a2)
    assert ra == ra2
    sim = prs.Sim(gp, phi0=to_dev(phi0))
    r1 = sim.step_n(13)
    r2 = sim.step_n(24)
    phi, dphi = sim.state()
    np.testing.assert_array_equal(host(phi), a)
    np.testing.assert_array_equal(host(dphi), pa)
    assert r1 + r2 == ra


def test_set_state_resume():
    """Resuming from a saved state is bitwise identical to a continuous run."""
    say("resume")
    shape = (200, 120)
    gp, _ = params_pair(shape, 0.25, m=1.0, W0=10.0, diag_every=5)
    phi0 = uniform_field(shape, 8)
    a, pa, ra, _ = gpu_run(gp, phi0, 30)
    prs = gpu_prs()
    s1 = prs.Sim(gp, phi0=to_dev(phi0))
    s1.step_n(17)
    phi, dphi = s1.state()
    s2 = prs.Sim(gp, phi0=to_dev(np.zeros(phi0.size)))
    s2.set_state(phi.clone(), dphi.clone(), 17)
    r = s2.step_n(13)
    np.testing.assert_array_equal(host(s2.state()[0]), a)
    assert r == [x for x in ra if x["step"] >= 17]


def test_nonfinite_detected():
    say("nonfinite")
    shape = (128, 64)
    gp, _ = params_pair(shape, 0.25, diag_every=1)
    phi0 = uniform_field(shape, 2).reshape(-1).copy()
    phi0[100] = np.nan
    phi0[2000] = np.inf
    prs = gpu_prs()
    sim = prs.Sim(gp, phi0=to_dev(phi0))
    st = sim.wall_stats()
    assert st["nonfinite"] == 2


def test_closed_form_diagnostics_on_gpu():
    """P10/P11 closed forms through the GPU diagnostics kernel."""
    say("closed-form diagnostics")
    prs = gpu_prs()
    shape = (64, 64)
    N = 64
    s = sum(F.coords(shape)) % N
    phi = np.where(s < N // 2, 0.7, -0.7)
    gp, _ = params_pair(shape, 0.25, W0=6.0)
    sim = prs.Sim(gp, phi0=to_dev(phi))
    assert sim.wall_stats()["area_density"] == pytest.approx(2.0 * math.sqrt(2) / N, rel=1e-14)
    W0, gv = 6.0, 0.7
    x = F.coords((128, 8))[0]
    prof = np.tanh(math.pi * (x - 31.5) / W0) * np.tanh(math.pi * (95.5 - x) / W0)
    prof32 = prof.astype(np.float32).astype(np.float64)
    dphi = -(gv / (W0 / math.pi)) * (1.0 - prof32 * prof32)
    gp, _ = params_pair((128, 8), 0.25, W0=W0)
    sim = prs.Sim(gp, phi0=to_dev(prof32), dphi0=to_dev(dphi))
    st = sim.wall_stats()
    # dphi is rounded to float32, so the ratio holds to ~1e-7
    assert st["gv2"] == pytest.approx(gv * gv, rel=1e-6)
    assert st["links"] == 2 * 8 and st["wall_sites"] == 4 * 8


# ------------------------------------------- full sizes (bench launch) -----

def default_tiling_of(sim):
    return sim.tiling()


@pytest.mark.parametrize("tiling,T", [((2, 64, 1), 8), ((2, 128, 1), 8), (None, None)])
def test_full_size_2d_8192_sampled(tiling, T):
    """8192^2 matter era in the launch configurations the benchmark's tuner
    picks (eight-step passes, 64 or 128 rows) and the library default:
    sampled patches after 64 steps match the oracle evolved on the patch's
    dependence cone; the full-lattice diagnostics match the oracle on the
    same field."""
    say("8192^2 full size", tiling, T)
    torch = torch_mod()
    prs = gpu_prs()
    shape = (8192, 8192)
    gp, op = params_pair(shape, 0.25, m=2.0, W0=10.0, diag_every=64)
    sim = prs.Sim(gp, seed=1)
    if tiling is not None:
        sim.set_tiling(*tiling)
        sim.set_time_blocking(T)
    say("  tiling", sim.tiling(), "steps/pass", sim.time_blocking())
    recs = sim.step_n(64)
    assert len(recs) == 1 and recs[0]["step"] == 0
    phi, dphi = sim.state()
    g = host(phi)
    gd = host(dphi)
    rng = np.random.default_rng(5)
    centers = [(0, 0), (8191, 8191), (4095, 17)] + [tuple(int(v) for v in rng.integers(0, 8192, 2))
                                                    for _ in range(5)]
    for c in centers:
        idx, ref = oracle_patch(op, shape, 1, c, 64, 6)
        assert rel_linf(g[idx], ref) <= 1e-5, c
    st = sim.wall_stats()
    o = O.stats(op, g.astype(np.float64), gd.astype(np.float64), 64)
    assert_stats_match(st, o, ctx="8192^2 n=64")
    # record of n = 0 equals the oracle on the seeded initial field
    phi0 = uniform_field(shape, 1).reshape(-1).astype(np.float64)
    assert_stats_match(recs[0], O.stats(op, phi0, np.zeros_like(phi0), 0), ctx="8192^2 n=0")
    del sim
    torch.cuda.empty_cache()


@pytest.mark.parametrize("tiling,T", [((2, 128, 1), 8), ((1, 64, 1), 1)])
def test_2d_lattice_past_2_32_sites(tiling, T):
    """A 65536 x 65600 lattice holds more than 2^32 sites, so row offsets of
    its last 64 rows exceed 32 bits: sampled patches there and elsewhere
    after 16 steps match the oracle on their dependence cones."""
    say("2D past 2^32 sites", tiling, T)
    torch = torch_mod()
    prs = gpu_prs()
    shape = (65536, 65600)
    assert shape[0] * shape[1] > 1 << 32
    gp, op = params_pair(shape, 0.25, m=2.0, W0=10.0)
    sim = prs.Sim(gp, seed=1)
    sim.set_tiling(*tiling)
    sim.set_time_blocking(T)
    sim.step_n(16, diag=False)
    phi, _ = sim.state()
    for c in [(0, 65599), (65535, 65590), (100, 65540), (40000, 65536), (30000, 32768), (5, 0)]:
        idx, ref = oracle_patch(op, shape, 1, c, 16, 5)
        got = host(phi.index_select(0, torch.from_numpy(idx).cuda()))
        assert rel_linf(got, ref) <= 1e-5, c
    del sim, phi
    torch.cuda.empty_cache()


@pytest.mark.parametrize("tiling,T", [((2, 64, 2), 3), (None, None)])
def test_full_size_3d_1024_sampled(tiling, T):
    """1024^3 radiation era in the fastest three-step configuration and the
    library default: sampled patches after 50 steps (one diagnostic interval)
    and the full-lattice diagnostics on the same field; the record of n = 0
    against the oracle on the seeded initial field."""
    say("1024^3 full size", tiling, T)
    torch = torch_mod()
    prs = gpu_prs()
    shape = (1024, 1024, 1024)
    gp, op = params_pair(shape, 0.2, m=1.0, W0=10.0, diag_every=50)
    sim = prs.Sim(gp, seed=1)
    if tiling is not None:
        sim.set_tiling(*tiling)
        sim.set_time_blocking(T)
    say("  tiling", sim.tiling(), "steps/pass", sim.time_blocking())
    recs = sim.step_n(50)
    assert len(recs) == 1 and recs[0]["step"] == 0
    phi, dphi = sim.state()
    rng = np.random.default_rng(6)
    centers = [(0, 0, 0), (1023, 1023, 1023), (511, 0, 1023)] + [
        tuple(int(v) for v in rng.integers(0, 1024, 3)) for _ in range(3)]
    pflat = phi.reshape(-1)
    for c in centers:
        idx, ref = oracle_patch(op, shape, 1, c, 50, 3)
        got = host(pflat[torch.from_numpy(idx).cuda()])
        assert rel_linf(got, ref) <= 1e-5, c
    st = sim.wall_stats()
    g = host(phi).astype(np.float64)
    gd = host(dphi).astype(np.float64)
    o = O.stats(op, g, gd, 50)
    assert_stats_match(st, o, ctx="1024^3 n=50")
    del g, gd
    phi0 = uniform_field(shape, 1).reshape(-1).astype(np.float64)
    assert_stats_match(recs[0], O.stats(op, phi0, np.zeros_like(phi0), 0), ctx="1024^3 n=0")
    del phi0, sim
    torch.cuda.empty_cache()


# --------------------------------------------------- multi-step passes ----

@pytest.mark.parametrize("shape,K,steps", [
    ((300, 70), 5, 23), ((1, 7), 2, 9), ((7, 1), 3, 10), ((2, 2), 64, 11), ((66, 129), 1, 6),
    ((1030, 9), 64, 67), ((256, 256), 10, 50), ((512, 300), 8, 37), ((248, 40), 12, 31),
    ((40, 30, 20), 5, 17), ((64, 9, 33), 8, 23), ((130, 6, 4), 3, 10), ((2, 3, 5), 64, 9),
    ((1, 1, 1), 2, 7), ((62, 17, 12), 1, 6),
])
def test_multi_step_passes_bitwise_equal_single_steps(shape, K, steps):
    """Temporal blocking (2D: 2, 3, 4, 6 or 8 steps per pass; 3D: 2 or 3)
    changes only how often HBM is visited: fields and records are bitwise
    those of single steps, for every tiling, ragged sizes, record cadences
    and odd step counts."""
    say("multi-step", shape, K, steps)
    prs = gpu_prs()
    deta = 0.25 if len(shape) == 2 else 0.2
    gp, _ = params_pair(shape, deta, m=2.0, W0=6.0, diag_every=K)
    phi0 = uniform_field(shape, 31)
    ref = prs.Sim(gp, phi0=to_dev(phi0))
    ref.set_time_blocking(1)
    r_ref = ref.step_n(steps)
    rp, rd = (host(t) for t in ref.state())
    base = tilings_for(shape)
    for T in ((2, 3, 4, 6, 8) if len(shape) == 2 else (2, 3)):
        for t in base + [(base[0][0], 8, 1)]:
            sim = prs.Sim(gp, phi0=to_dev(phi0))
            sim.set_time_blocking(T)
            sim.set_tiling(*t)
            r1 = sim.step_n(steps // 2)
            r2 = sim.step_n(steps - steps // 2)
            p, d = (host(x) for x in sim.state())
            np.testing.assert_array_equal(p, rp, err_msg=str((T, t)))
            np.testing.assert_array_equal(d, rd, err_msg=str((T, t)))
            assert [r["step"] for r in r1 + r2] == [r["step"] for r in r_ref]
            for a, b in zip(r1 + r2, r_ref):
                assert_stats_match(a, b, rel=1e-13, ctx=str((T, t)))
            assert sim.state()[1].data_ptr() == sim.dphi.data_ptr()


@pytest.mark.parametrize("shape,K,steps", [
    ((40, 30, 20), 5, 17), ((64, 9, 33), 8, 23), ((130, 6, 4), 3, 10), ((2, 3, 5), 64, 9),
    ((1, 1, 1), 2, 7), ((62, 41, 12), 1, 6), ((128, 70, 45), 10, 26),
])
def test_lds_pass_bitwise_equal_single_steps(shape, K, steps):
    """The LDS-staged 3D pass (a workgroup of waves stacked along y, row
    halos shared through LDS; ty 8, 16: eight waves of 2, 4 rows; ty 32, 64:
    sixteen waves of 2, 4 rows) with 2, 3 and 4 steps per pass, one and two
    sites per lane: fields and record
    counts bit for bit those of single steps, the FP64 record sums to
    summation order, for lattices thinner than a workgroup's rows, ragged
    row and plane tiles and split calls."""
    say("lds pass", shape, K, steps)
    prs = gpu_prs()
    gp, _ = params_pair(shape, 0.2, m=2.0, W0=6.0, diag_every=K)
    phi0 = uniform_field(shape, 32)
    ref = prs.Sim(gp, phi0=to_dev(phi0))
    ref.set_time_blocking(1)
    r_ref = ref.step_n(steps)
    rp, rd = (host(t) for t in ref.state())
    for T in (2, 3, 4):
        for vec in (1, 2):
            if shape[0] % vec:
                continue
            for t in ((vec, 8, 8), (vec, 13, 16), (vec, 64, 16), (vec, 9, 8), (vec, 11, 32)) + \
                    (((vec, 9, 64),) if vec == 1 else ()):
                sim = prs.Sim(gp, phi0=to_dev(phi0))
                sim.set_tiling(*t)
                sim.set_time_blocking(T)
                r1 = sim.step_n(steps // 2)
                r2 = sim.step_n(steps - steps // 2)
                p, d = (host(x) for x in sim.state())
                np.testing.assert_array_equal(p, rp, err_msg=str((T, t)))
                np.testing.assert_array_equal(d, rd, err_msg=str((T, t)))
                assert [r["step"] for r in r1 + r2] == [r["step"] for r in r_ref]
                for a, b in zip(r1 + r2, r_ref):
                    assert_stats_match(a, b, rel=1e-13, ctx=str((T, t)))


def test_lds_pass_f64():
    """The LDS-staged 3D pass in float64 (one site per lane), T = 2, 3, 4."""
    say("lds pass f64")
    prs = gpu_prs()
    shape = (48, 37, 20)
    gp = prs.make_params(shape, deta=0.2, m=1.0, W0=6.0, diag_every=7, precision=prs.PRS_F64)
    ref = prs.Sim(gp, seed=33)
    ref.set_time_blocking(1)
    r_ref = ref.step_n(19)
    rp, rd = (host(t) for t in ref.state())
    for T in (2, 3, 4):
        for t in ((1, 8, 8), (1, 16, 16)):
            sim = prs.Sim(gp, seed=33)
            sim.set_tiling(*t)
            sim.set_time_blocking(T)
            recs = sim.step_n(19)
            p, d = (host(x) for x in sim.state())
            np.testing.assert_array_equal(p, rp, err_msg=str((T, t)))
            np.testing.assert_array_equal(d, rd, err_msg=str((T, t)))
            for a, b in zip(recs, r_ref):
                assert_stats_match(a, b, rel=1e-13, ctx=str((T, t)))


def test_multi_step_default_and_limits():
    prs = gpu_prs()
    gp, _ = params_pair((64, 64), 0.25)
    sim = prs.Sim(gp, seed=1)
    assert sim.time_blocking() == 2
    for bad in (5, 7, 9, 0):
        with pytest.raises(prs.PRSError) as e:
            sim.set_time_blocking(bad)
        assert e.value.status == prs.PRS_EINVAL
    gp64 = prs.make_params((64, 64), deta=0.25, precision=prs.PRS_F64)
    sim64 = prs.Sim(gp64, seed=1)
    sim64.set_time_blocking(4)
    sim64.set_time_blocking(8)          # float64 eight-step passes run with vec 1
    with pytest.raises(prs.PRSError) as e:
        sim64.set_time_blocking(5)
    assert e.value.status == prs.PRS_EINVAL
    gp3, _ = params_pair((16, 16, 16), 0.2)
    sim3 = prs.Sim(gp3, seed=1)
    assert sim3.time_blocking() == 1
    sim3.set_time_blocking(3)
    sim3.set_time_blocking(4)           # the LDS-staged pass (ty 8, 16) runs four steps
    for bad in (5, 6, 8):
        with pytest.raises(prs.PRSError) as e:
            sim3.set_time_blocking(bad)
        assert e.value.status == prs.PRS_EINVAL
    gp364 = prs.make_params((16, 16, 16), deta=0.2, precision=prs.PRS_F64)
    sim364 = prs.Sim(gp364, seed=1)
    sim364.set_time_blocking(2)
    sim364.set_time_blocking(4)
    with pytest.raises(prs.PRSError) as e:
        sim364.set_time_blocking(5)
    assert e.value.status == prs.PRS_EINVAL


@pytest.mark.parametrize("shape,T,tiling", [((8192, 8192), 8, (2, 64, 1)), ((8192, 8192), 8, (2, 128, 1)),
                                            ((1024, 1024, 1024), 3, (1, 16, 4)), ((1024, 1024, 1024), 3, (2, 64, 2)),
                                            ((1024, 1024, 1024), 2, (2, 32, 1))])
def test_full_size_multi_step_bitwise(shape, T, tiling):
    """At the full lattice sizes the multi-step passes reproduce single steps
    bit for bit (fields compared on the device) and their fused record
    equals the single-step record up to summation order."""
    say("full-size multi-step", shape, T, tiling)
    torch = torch_mod()
    prs = gpu_prs()
    deta = 0.25 if len(shape) == 2 else 0.2
    gp, _ = params_pair(shape, deta, m=1.0, W0=10.0, diag_every=6)
    steps = 2 * T
    ref = prs.Sim(gp, seed=1)
    ref.set_tiling(*tiling)
    ref.set_time_blocking(1)
    r_ref = ref.step_n(steps)
    sim = prs.Sim(gp, seed=1)
    sim.set_tiling(*tiling)
    sim.set_time_blocking(T)
    assert prs.prs_plan_passes(sim.ctx, steps)[0] >= 1
    r = sim.step_n(steps)
    for a, b in zip(sim.state(), ref.state()):
        assert torch.equal(a, b)
    for a, b in zip(r, r_ref):
        assert_stats_match(a, b, rel=1e-12, ctx="full-size multi-step")
    del ref, sim
    torch.cuda.empty_cache()
