"""Batched ensemble: every realisation inside the batch reproduces the same
realisation run alone (fields, counts and records bit for bit with the same
tiling and steps per pass), for uneven sizes, dimensions, eras and step
counts, in every launch mode (the persistent kernel in one launch with and
without a graph and in one launch per phase, concurrent streams with and
without a graph), across graph replays and mode switches; and every member's
evolved field against the oracle's run of the same realisation."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1710_10420_amd.inputs import uniform_field
from tests.gpu_util import assert_stats_match, gpu_prs, host, say, torch_mod

pytestmark = pytest.mark.gpu

SPECS = [
    dict(shape=(256, 256), deta=0.25, m=0.5, W0=5.0, nsteps=50, diag_every=10, seed=1000),
    dict(shape=(300, 70), deta=0.25, m=1.0, W0=10.0, nsteps=37, diag_every=8, seed=1001),
    dict(shape=(512, 512), deta=0.25, m=2.0, W0=10.0, nsteps=80, diag_every=16, seed=1002),
    dict(shape=(40, 30, 20), deta=0.2, m=1.0, W0=5.0, nsteps=23, diag_every=5, seed=1003),
    dict(shape=(64, 64, 64), deta=0.2, m=0.5, W0=10.0, nsteps=31, diag_every=10, seed=1004),
    dict(shape=(33, 17), deta=0.25, m=1.0, W0=5.0, nsteps=0, diag_every=4, seed=1005),
    dict(shape=(128, 96), deta=0.25, m=1.0, W0=10.0, nsteps=1, diag_every=1, seed=1006),
    dict(shape=(200, 64), deta=0.25, m=1.0, W0=10.0, nsteps=29, diag_every=7, seed=1007, T=1),
]

TILINGS = [(4, 32, 1), (2, 17, 1), (4, 64, 1), (2, 16, 1), (4, 32, 1), (1, 16, 1), (4, 8, 1), (2, 16, 1)]


def steps_per_pass(sp):
    return sp.get("T", 2 if len(sp["shape"]) == 2 else 1)


def single_run(prs, sp, tiling):
    p = prs.make_params(sp["shape"], deta=sp["deta"], m=sp["m"], W0=sp["W0"],
                        diag_every=sp["diag_every"])
    sim = prs.Sim(p, seed=sp["seed"])
    sim.set_tiling(*tiling)
    sim.set_time_blocking(steps_per_pass(sp))
    recs = sim.step_n(sp["nsteps"])
    recs.append(sim.wall_stats())
    phi, dphi = sim.state()
    return host(phi), host(dphi), recs


@pytest.fixture(scope="module")
def singles():
    prs = gpu_prs()
    out = []
    for sp, t in zip(SPECS, TILINGS):
        say("single", sp["shape"], sp["nsteps"])
        out.append(single_run(prs, sp, t))
    return out


def make_batch(prs):
    b = prs.Batch(SPECS)
    for r, t in enumerate(TILINGS):
        b.set_tiling(r, *t)
        b.set_time_blocking(r, steps_per_pass(SPECS[r]))
    return b


@pytest.mark.parametrize("mode", [0, 1, 2, 3, 4])
def test_batch_equals_single_runs(singles, mode):
    say("batch mode", mode)
    prs = gpu_prs()
    b = make_batch(prs)
    b.set_mode(mode)
    for rep in range(2):                 # the graph is replayed on the second run
        recs = b.run()
        for r, sp in enumerate(SPECS):
            phi, dphi = b.final_state(r)
            s_phi, s_dphi, s_recs = singles[r]
            np.testing.assert_array_equal(host(phi), s_phi)
            np.testing.assert_array_equal(host(dphi), s_dphi)
            assert recs[r] == s_recs, (mode, rep, r)
    b.close()


def test_batch_records_match_oracle_on_final_state(singles):
    """Final-state records of the ensemble equal the oracle diagnostics of
    that state (counts bitwise)."""
    say("batch vs oracle")
    prs = gpu_prs()
    b = make_batch(prs)
    recs = b.run()
    for r, sp in enumerate(SPECS):
        phi, dphi = b.final_state(r)
        op = O.params(sp["shape"], deta=sp["deta"], m=sp["m"], W0=sp["W0"])
        o = O.stats(op, host(phi).astype(np.float64), host(dphi).astype(np.float64), sp["nsteps"])
        assert_stats_match(recs[r][-1], o, ctx=str(sp["shape"]))
    b.close()


def test_batch_fields_match_oracle(singles):
    """Every member's evolved field, run inside the ensemble, against the
    oracle's run of the same realisation (its seed, size, era, width and
    step count): relative L-inf <= 1e-5, and the records the ensemble wrote
    along the way against the oracle's records of its own trajectory (counts
    bit for bit while the float32 and float64 trajectories still give the
    same signs, which at these lengths they do)."""
    say("batch fields vs oracle")
    prs = gpu_prs()
    from tests.gpu_util import rel_linf
    b = make_batch(prs)
    recs = b.run()
    for r, sp in enumerate(SPECS):
        phi, dphi = b.final_state(r)
        op = O.params(sp["shape"], deta=sp["deta"], m=sp["m"], W0=sp["W0"])
        phi0 = uniform_field(sp["shape"], sp["seed"]).astype(np.float64).reshape(-1)
        ophi, opi, orecs = O.run(op, phi0, np.zeros_like(phi0), sp["nsteps"], diag_every=sp["diag_every"])
        if sp["nsteps"] > 0:
            assert rel_linf(host(phi), ophi) <= 1e-5, sp
            assert rel_linf(host(dphi), opi) <= 1e-5, sp
        else:
            np.testing.assert_array_equal(host(phi).astype(np.float64), ophi)
        assert len(recs[r]) == len(orecs) + 1, sp
        for g, o in zip(recs[r], orecs):
            assert g["links_dir"] == o["links_dir"] and g["wall_sites"] == o["wall_sites"], (sp, g["step"])
            assert g["area_density"] == pytest.approx(o["area_density"], rel=1e-5)
    b.close()


def test_batch_initial_fields_from_seeds():
    prs = gpu_prs()
    sp = dict(shape=(100, 60), deta=0.25, m=1.0, W0=10.0, nsteps=0, diag_every=1, seed=77)
    b = prs.Batch([sp])
    b.run()
    phi, dphi = b.final_state(0)
    np.testing.assert_array_equal(host(phi), uniform_field((100, 60), 77).reshape(-1))
    assert float(host(dphi).max()) == 0.0 and float(host(dphi).min()) == 0.0
    b.close()


def test_batch_rejects_invalid_item():
    prs = gpu_prs()
    bad = dict(SPECS[0])
    bad["deta"] = 2.0
    with pytest.raises(prs.PRSError) as e:
        prs.Batch([SPECS[1], bad])
    assert e.value.status == prs.PRS_EINVAL and "item 1" in str(e.value)


# Settings only the stream modes run: 3 and 4 steps per pass in 2D, 3D tiles
# of 2 and 4 rows.
SPECS_WIDE = [
    dict(shape=(256, 256), deta=0.25, m=0.5, W0=5.0, nsteps=50, diag_every=10, seed=2000, T=4),
    dict(shape=(300, 70), deta=0.25, m=1.0, W0=10.0, nsteps=37, diag_every=8, seed=2001, T=3),
    dict(shape=(40, 30, 20), deta=0.2, m=1.0, W0=5.0, nsteps=23, diag_every=5, seed=2002),
    dict(shape=(64, 64, 64), deta=0.2, m=0.5, W0=10.0, nsteps=31, diag_every=10, seed=2003),
    dict(shape=(512, 128), deta=0.25, m=2.0, W0=10.0, nsteps=61, diag_every=0, seed=2004, T=4),
    dict(shape=(96, 90), deta=0.25, m=1.0, W0=10.0, nsteps=9, diag_every=3, seed=2005, T=4),
]
TILINGS_WIDE = [(1, 16, 1), (2, 8, 1), (2, 16, 2), (1, 32, 4), (4, 16, 1), (2, 8, 1)]


@pytest.fixture(scope="module")
def singles_wide():
    prs = gpu_prs()
    out = []
    for sp, t in zip(SPECS_WIDE, TILINGS_WIDE):
        say("single", sp["shape"], sp["nsteps"], t, steps_per_pass(sp))
        out.append(single_run(prs, sp, t))
    return out


@pytest.mark.parametrize("mode", [3, 4])
def test_stream_modes_wide_settings(singles_wide, mode):
    say("stream batch mode", mode)
    prs = gpu_prs()
    b = prs.Batch(SPECS_WIDE)
    for r, t in enumerate(TILINGS_WIDE):
        b.set_tiling(r, *t)
        b.set_time_blocking(r, steps_per_pass(SPECS_WIDE[r]))
    b.set_mode(mode)
    for rep in range(3):
        recs = b.run()
        for r in range(len(SPECS_WIDE)):
            phi, dphi = b.final_state(r)
            s_phi, s_dphi, s_recs = singles_wide[r]
            np.testing.assert_array_equal(host(phi), s_phi)
            np.testing.assert_array_equal(host(dphi), s_dphi)
            if SPECS_WIDE[r]["diag_every"] > 0:
                assert recs[r] == s_recs, (mode, rep, r)
            else:
                assert recs[r] == s_recs[-1:], (mode, rep, r)
    b.close()


# Multi-step settings of the persistent kernel: 2D eight-, six-, four- and
# three-step passes (records on and off pass boundaries, ragged tiles), and
# 3D LDS-staged passes of four and three steps with workgroups of eight
# waves of 2 or 4 rows, next to 3D single steps.
SPECS_PK = [
    dict(shape=(256, 256), deta=0.25, m=0.5, W0=5.0, nsteps=70, diag_every=16, seed=3000, T=8),
    dict(shape=(300, 70), deta=0.25, m=1.0, W0=10.0, nsteps=45, diag_every=10, seed=3001, T=8),
    dict(shape=(200, 96), deta=0.25, m=2.0, W0=10.0, nsteps=40, diag_every=0, seed=3002, T=6),
    dict(shape=(128, 100), deta=0.25, m=1.0, W0=5.0, nsteps=29, diag_every=7, seed=3003, T=4),
    dict(shape=(96, 90), deta=0.25, m=1.0, W0=10.0, nsteps=23, diag_every=9, seed=3004, T=3),
    dict(shape=(64, 64, 64), deta=0.2, m=0.5, W0=10.0, nsteps=33, diag_every=12, seed=3005, T=4),
    dict(shape=(40, 30, 20), deta=0.2, m=1.0, W0=5.0, nsteps=25, diag_every=5, seed=3006, T=3),
    dict(shape=(48, 56, 40), deta=0.2, m=1.0, W0=10.0, nsteps=19, diag_every=6, seed=3007, T=4),
    dict(shape=(32, 32, 24), deta=0.2, m=2.0, W0=5.0, nsteps=11, diag_every=4, seed=3008, T=1),
    dict(shape=(33, 17), deta=0.25, m=1.0, W0=5.0, nsteps=0, diag_every=4, seed=3009, T=8),
]
TILINGS_PK = [(2, 16, 1), (2, 8, 1), (1, 32, 1), (4, 16, 1), (4, 8, 1), (1, 16, 8), (1, 8, 16), (1, 12, 8),
              (2, 8, 1), (1, 8, 1)]


@pytest.fixture(scope="module")
def singles_pk():
    prs = gpu_prs()
    out = []
    for sp, t in zip(SPECS_PK, TILINGS_PK):
        say("single", sp["shape"], sp["nsteps"], t, steps_per_pass(sp))
        out.append(single_run(prs, sp, t))
    return out


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_persistent_multi_step_settings(singles_pk, mode):
    """The persistent kernel with multi-step passes (2D up to eight steps,
    3D LDS-staged passes up to four): every realisation bit for bit its
    single run, records included, across graph replays."""
    say("persistent batch mode", mode)
    prs = gpu_prs()
    b = prs.Batch(SPECS_PK)
    for r, t in enumerate(TILINGS_PK):
        b.set_tiling(r, *t)
        b.set_time_blocking(r, steps_per_pass(SPECS_PK[r]))
    b.set_mode(mode)
    for rep in range(3):
        recs = b.run()
        for r in range(len(SPECS_PK)):
            phi, dphi = b.final_state(r)
            s_phi, s_dphi, s_recs = singles_pk[r]
            np.testing.assert_array_equal(host(phi), s_phi)
            np.testing.assert_array_equal(host(dphi), s_dphi)
            if SPECS_PK[r]["diag_every"] > 0:
                assert recs[r] == s_recs, (mode, rep, r)
            else:
                assert recs[r] == s_recs[-1:], (mode, rep, r)
    b.close()


def test_persistent_modes_reject_other_settings():
    """Settings the persistent kernel holds no code for are refused before
    any launch, naming the item: 2D vec 4 beyond four steps per pass, the
    one-wave 3D tilings with ty 2 or 4, 3D ty 16 at four steps per pass and
    float64 items."""
    prs = gpu_prs()
    b = prs.Batch(SPECS_WIDE[:4])
    b.set_mode(prs.PRS_BATCH_PERSISTENT)
    b.set_tiling(0, 4, 16, 1)
    b.set_time_blocking(0, 8)
    with pytest.raises(prs.PRSError) as e:
        b.run()
    assert e.value.status == prs.PRS_EINVAL and "item 0" in str(e.value)
    b.set_time_blocking(0, 4)
    b.set_tiling(2, 2, 16, 2)
    b.set_time_blocking(2, 1)
    with pytest.raises(prs.PRSError) as e:
        b.run()
    assert e.value.status == prs.PRS_EINVAL and "item 2" in str(e.value)
    b.set_tiling(2, 1, 8, 16)
    b.set_time_blocking(2, 4)
    with pytest.raises(prs.PRSError) as e:
        b.run()
    assert e.value.status == prs.PRS_EINVAL and "item 2" in str(e.value)
    b.set_time_blocking(2, 3)
    b.set_tiling(3, 1, 8, 8)
    b.set_time_blocking(3, 4)
    b.run()
    b.close()
    f64 = [dict(SPECS_WIDE[0], precision=prs.PRS_F64)]
    b = prs.Batch(f64)
    b.set_mode(prs.PRS_BATCH_PERSISTENT)
    with pytest.raises(prs.PRSError) as e:
        b.run()
    assert e.value.status == prs.PRS_EINVAL and "item 0" in str(e.value)
    b.close()


def test_mode_switches_keep_results(singles):
    """Stream, persistent and graph modes in turn on one ensemble: each run
    reproduces the single runs."""
    say("batch mode switches")
    prs = gpu_prs()
    b = make_batch(prs)
    for mode in (4, 0, 3, 1, 3, 2, 0):
        b.set_mode(mode)
        recs = b.run()
        for r in range(len(SPECS)):
            phi, dphi = b.final_state(r)
            s_phi, s_dphi, s_recs = singles[r]
            np.testing.assert_array_equal(host(phi), s_phi)
            np.testing.assert_array_equal(host(dphi), s_dphi)
            assert recs[r] == s_recs, (mode, r)
    b.close()


@pytest.mark.parametrize("mode", [0, 2, 4])
def test_batch_autotune_keeps_results(singles_pk, mode):
    """The ensemble-level tuner only lengthens marching tiles (doubling,
    up to 128) and, for 3D workgroup-stacked tilings, changes the workgroup
    shape and steps per pass; vec, and in 2D ty and steps per pass, stay.
    Afterwards every realisation's field is still bit for bit its single run
    (fields depend on neither tiling nor steps per pass), its counts too,
    and its two floating-point means equal up to summation order."""
    say("batch autotune mode", mode)
    prs = gpu_prs()
    specs = SPECS_PK if mode != 4 else SPECS_PK[:5]
    b = prs.Batch(specs)
    for r in range(len(specs)):
        b.set_tiling(r, *TILINGS_PK[r])
        b.set_time_blocking(r, steps_per_pass(specs[r]))
    b.set_mode(mode)
    ms = b.autotune()
    assert ms > 0.0
    for r in range(len(specs)):
        (vec, rows, ty), T = b.tiling(r)
        v0, r0, t0 = TILINGS_PK[r]
        if len(specs[r]["shape"]) == 3 and t0 >= 8 and steps_per_pass(specs[r]) > 1:
            assert vec == v0 and ty in (8, 16, 32, 64) and T in (2, 3, 4), (r, ty, T)
        else:
            assert (vec, ty, T) == (v0, t0, steps_per_pass(specs[r])), r
        assert rows >= r0 and rows % r0 == 0 and (rows // r0) & (rows // r0 - 1) == 0, (r, rows)
        assert rows == r0 or rows <= 128, (r, rows)
    for rep in range(2):
        recs = b.run()
        for r in range(len(specs)):
            phi, dphi = b.final_state(r)
            s_phi, s_dphi, s_recs = singles_pk[r]
            np.testing.assert_array_equal(host(phi), s_phi)
            np.testing.assert_array_equal(host(dphi), s_dphi)
            want = s_recs if specs[r]["diag_every"] > 0 else s_recs[-1:]
            assert len(recs[r]) == len(want), r
            for g, o in zip(recs[r], want):
                for k in ("step", "eta", "links", "links_dir", "wall_sites", "nonfinite"):
                    assert g[k] == o[k], (r, k)
                assert g["area_density"] == pytest.approx(o["area_density"], rel=1e-12, abs=1e-300)
                assert g["gv2"] == pytest.approx(o["gv2"], rel=1e-12, abs=1e-300)
    b.close()


def test_batch_autotune_requires_seeded_items():
    """The ensemble tuner reruns the ensemble, so it refuses an ensemble
    whose items start from their buffers' contents (before any launch)."""
    prs = gpu_prs()
    torch = torch_mod()
    b = prs.Batch(SPECS[:2])
    items = []
    for it in b.items:
        c = prs.prs_batch_item.from_buffer_copy(it)
        c.init_from_seed = 0
        items.append(c)
    nb = prs.prs_batch_workspace_bytes(items)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    h = prs.prs_batch_create(items, ws.data_ptr(), nb, prs._stream_handle(torch.cuda.current_stream()))
    try:
        with pytest.raises(prs.PRSError) as e:
            prs.prs_batch_autotune(h)
        assert e.value.status == prs.PRS_EINVAL and "item 0" in str(e.value)
    finally:
        prs.prs_batch_destroy(h)
    b.close()
