"""Slab passes: the per-device kernel of a lattice sharded along its last
axis (y in 2D, z in 3D).  A slab stored with T halo rows or planes below and
above, filled here with the periodic images a neighbouring device would
send, must advance its interior exactly as the whole periodic lattice does
(same kernel arithmetic, so bitwise), for both precisions and the physical
force."""
import numpy as np
import pytest

from tests.gpu_util import gpu_prs, host, say, torch_mod

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,T,tiling,nslab,f64,beta", [
    ((96, 64), 8, (2, 16, 1), 2, False, 0.0),
    ((80, 60), 3, (1, 8, 1), 3, False, 2.0),
    ((72, 48), 4, (4, 8, 1), 2, False, 0.0),
    ((40, 36), 6, (1, 8, 1), 2, True, 0.0),
    ((48, 32), 8, (1, 16, 1), 2, True, 2.0),
    ((64, 12), 8, (1, 8, 1), 4, False, 0.0),      # slabs of 3 rows, thinner than their halos
    ((64, 40, 32), 3, (1, 8, 2), 2, False, 0.0),
    ((48, 36, 30), 2, (2, 8, 1), 3, False, 0.0),
    ((48, 36, 30), 3, (1, 8, 4), 3, False, 2.0),
    ((40, 24, 20), 2, (1, 8, 2), 2, True, 0.0),
    ((32, 16, 8), 3, (1, 8, 1), 4, False, 0.0),   # slabs of 2 planes, thinner than their halos
    ((64, 40, 32), 4, (2, 8, 16), 2, False, 0.0),  # the LDS-staged pass (eight waves of four rows)
    ((48, 36, 30), 3, (1, 8, 8), 3, False, 2.0),   # eight waves of two rows
    ((40, 24, 20), 4, (1, 8, 8), 2, True, 0.0),
    ((48, 44, 24), 4, (1, 8, 64), 3, False, 0.0),  # sixteen waves of four rows, slabs of 8 planes
])
def test_slab_passes_equal_the_whole_lattice(shape, T, tiling, nslab, f64, beta):
    torch = torch_mod()
    prs = gpu_prs()
    say("slab", shape, T, tiling, nslab, f64, beta)
    lay = tuple(reversed(shape))                    # (z,) y, x
    NZ, plane = lay[0], lay[1:]
    kw = dict(deta=0.2 if beta == 0.0 else 0.1, m=1.0, W0=8.0, alpha=3.0 if beta == 0.0 else 2.0, beta=beta,
              precision=prs.PRS_F64 if f64 else prs.PRS_F32)
    gp = prs.make_params(shape, **kw)
    sim = prs.Sim(gp, seed=4)
    sim.set_time_blocking(1)
    sim.step_n(5)                                   # phi_dot != 0 from here
    phi5, pi5 = (t.clone() for t in sim.state())
    sim.set_tiling(*tiling)
    sim.set_time_blocking(T)
    sim.step_n(T)
    ref_phi, ref_pi = (host(t).reshape(lay) for t in sim.state())
    nz = NZ // nslab
    stream = prs._stream_handle(torch.cuda.current_stream())
    for sl in range(nslab):
        z0 = sl * nz
        planes = torch.tensor([(z0 - T + k) % NZ for k in range(nz + 2 * T)], device="cuda")
        phi_in = phi5.view(lay).index_select(0, planes).contiguous()
        pi_in = pi5.view(lay).index_select(0, planes).contiguous()
        phi_out = torch.zeros_like(phi_in)
        pi_out = torch.zeros_like(pi_in)
        ps = prs.make_params(tuple(shape[:-1]) + (nz,), **kw)
        prs.prs_slab_pass(ps, 5, T, tiling, phi_in.data_ptr(), phi_out.data_ptr(), pi_in.data_ptr(),
                          pi_out.data_ptr(), stream)
        torch.cuda.synchronize()
        got_phi = host(phi_out).reshape((nz + 2 * T,) + plane)
        got_pi = host(pi_out).reshape((nz + 2 * T,) + plane)
        np.testing.assert_array_equal(got_phi[T:T + nz], ref_phi[z0:z0 + nz], err_msg=str(sl))
        np.testing.assert_array_equal(got_pi[T:T + nz], ref_pi[z0:z0 + nz], err_msg=str(sl))
        # the halo rows or planes of the outputs are left alone
        assert not np.any(got_phi[:T]) and not np.any(got_phi[T + nz:])
        assert not np.any(got_pi[:T]) and not np.any(got_pi[T + nz:])


def test_slab_pass_rejects_bad_arguments():
    torch = torch_mod()
    prs = gpu_prs()
    stream = prs._stream_handle(torch.cuda.current_stream())
    bufs = [torch.zeros(32 * 16 * 14, device="cuda") for _ in range(4)]
    ptrs = [b.data_ptr() for b in bufs]
    p3 = prs.make_params((32, 16, 10), deta=0.2)
    p2 = prs.make_params((32, 16), deta=0.2)
    for args in ((p2, 0, 2, (1, 8, 2)), (p2, 0, 5, (1, 8, 1)), (p3, 0, 4, (1, 8, 2)), (p3, -1, 2, (1, 8, 2)),
                 (p3, 0, 2, (4, 8, 2))):
        with pytest.raises(prs.PRSError) as e:
            prs.prs_slab_pass(*args, *ptrs, stream)
        assert e.value.status == prs.PRS_EINVAL
    with pytest.raises(prs.PRSError) as e:
        prs.prs_slab_pass(p3, 0, 2, (1, 8, 2), ptrs[0], ptrs[0], ptrs[2], ptrs[3], stream)
    assert e.value.status == prs.PRS_EINVAL


@pytest.mark.parametrize("shape,T,tiling,nslab", [
    ((8192, 8192), 8, (2, 64, 1), 8),
    ((1024, 1024, 1024), 3, (2, 64, 2), 8),
])
def test_slab_full_size_in_the_benchmark_configurations(shape, T, tiling, nslab):
    """The slabs the benchmark times (one eighth of 8192^2 along y, eight-step
    passes; one eighth of 1024^3 along z, three-step passes), in its launch
    configurations: every slab of the whole lattice advances bit for bit as
    the whole lattice does, and the slabs' records of the input state combine
    into the whole lattice's record."""
    torch = torch_mod()
    prs = gpu_prs()
    say("slab full size", shape, T, tiling, nslab)
    kw = dict(deta=0.25, m=2.0, W0=10.0) if len(shape) == 2 else dict(deta=0.2, m=1.0, W0=10.0)
    lay = tuple(reversed(shape))
    NZ = lay[0]
    gp = prs.make_params(shape, **kw)
    sim = prs.Sim(gp, seed=1)
    sim.set_time_blocking(1)
    sim.step_n(3, diag=False)                       # phi_dot != 0 from here
    whole = sim.wall_stats()
    phi3, pi3 = (t.clone() for t in sim.state())
    sim.set_tiling(*tiling)
    sim.set_time_blocking(T)
    sim.step_n(T, diag=False)
    ref_phi, ref_pi = (t.view(lay) for t in sim.state())
    nz = NZ // nslab
    stream = prs._stream_handle(torch.cuda.current_stream())
    ps = prs.make_params(tuple(shape[:-1]) + (nz,), **kw)
    nb = prs.prs_slab_scratch_bytes(ps, T, tiling)
    scratch = torch.empty(nb, dtype=torch.uint8, device="cuda")
    sites = gp.n[0] * gp.n[1] * (gp.n[2] if len(shape) == 3 else 1) // nslab
    links, walls, area, ek = 0, 0, 0.0, 0.0
    for sl in range(nslab):
        z0 = sl * nz
        planes = torch.tensor([(z0 - T + k) % NZ for k in range(nz + 2 * T)], device="cuda")
        phi_in = phi3.view(lay).index_select(0, planes).contiguous()
        pi_in = pi3.view(lay).index_select(0, planes).contiguous()
        phi_out = torch.zeros_like(phi_in)
        pi_out = torch.zeros_like(pi_in)
        rec = prs.prs_slab_pass_stats(ps, 3, T, tiling, phi_in.data_ptr(), phi_out.data_ptr(), pi_in.data_ptr(),
                                      pi_out.data_ptr(), scratch.data_ptr(), nb, stream)
        assert torch.equal(phi_out[T:T + nz], ref_phi[z0:z0 + nz]), sl
        assert torch.equal(pi_out[T:T + nz], ref_pi[z0:z0 + nz]), sl
        links += rec["links"]
        walls += rec["wall_sites"]
        area += rec["area_density"] * sites
        ek += rec["gv2"] * rec["wall_sites"]
        del phi_in, pi_in, phi_out, pi_out
    assert links == whole["links"] and walls == whole["wall_sites"] > 0
    assert abs(area / (sites * nslab) - whole["area_density"]) <= 1e-12 * whole["area_density"]
    assert abs(ek / walls - whole["gv2"]) <= 1e-12 * whole["gv2"]
    del sim, phi3, pi3, ref_phi, ref_pi
    torch.cuda.empty_cache()


@pytest.mark.parametrize("shape,T,tiling,nslab,f64,beta", [
    ((96, 64), 8, (2, 16, 1), 2, False, 0.0),
    ((80, 60), 3, (1, 8, 1), 3, False, 2.0),
    ((40, 36), 6, (1, 8, 1), 2, True, 0.0),
    ((64, 40, 32), 3, (1, 8, 2), 2, False, 0.0),
    ((48, 36, 30), 3, (1, 8, 4), 3, False, 2.0),
    ((40, 24, 20), 2, (1, 8, 2), 2, True, 0.0),
    ((64, 40, 32), 4, (2, 8, 16), 2, False, 0.0),
    ((40, 24, 20), 3, (1, 8, 8), 2, True, 2.0),
])
def test_slab_pass_stats_add_up_to_the_whole_lattice(shape, T, tiling, nslab, f64, beta):
    """The slabs' records of their input state combine into the whole
    lattice's record of the same state: counts bit for bit, the area per
    site and the wall-site mean of (gamma v)^2 to summation-order rounding;
    the fields advance exactly as without diagnostics."""
    torch = torch_mod()
    prs = gpu_prs()
    say("slab stats", shape, T, tiling, nslab, f64, beta)
    lay = tuple(reversed(shape))
    NZ, plane = lay[0], lay[1:]
    kw = dict(deta=0.2 if beta == 0.0 else 0.1, m=1.0, W0=8.0, alpha=3.0 if beta == 0.0 else 2.0, beta=beta,
              precision=prs.PRS_F64 if f64 else prs.PRS_F32)
    gp = prs.make_params(shape, **kw)
    sim = prs.Sim(gp, seed=4)
    sim.set_time_blocking(1)
    sim.step_n(5)
    whole = sim.wall_stats()
    phi5, pi5 = (t.clone() for t in sim.state())
    sim.set_tiling(*tiling)
    sim.set_time_blocking(T)
    sim.step_n(T)
    ref_phi, ref_pi = (host(t).reshape(lay) for t in sim.state())
    nz = NZ // nslab
    stream = prs._stream_handle(torch.cuda.current_stream())
    ps = prs.make_params(tuple(shape[:-1]) + (nz,), **kw)
    nb = prs.prs_slab_scratch_bytes(ps, T, tiling)
    assert nb > 0
    scratch = torch.empty(nb, dtype=torch.uint8, device="cuda")
    sites = nz
    for n in plane:
        sites *= n
    links = links_dir = None
    walls = nonfinite = 0
    area = ek = 0.0
    for sl in range(nslab):
        z0 = sl * nz
        planes = torch.tensor([(z0 - T + k) % NZ for k in range(nz + 2 * T)], device="cuda")
        phi_in = phi5.view(lay).index_select(0, planes).contiguous()
        pi_in = pi5.view(lay).index_select(0, planes).contiguous()
        phi_out = torch.zeros_like(phi_in)
        pi_out = torch.zeros_like(pi_in)
        rec = prs.prs_slab_pass_stats(ps, 5, T, tiling, phi_in.data_ptr(), phi_out.data_ptr(), pi_in.data_ptr(),
                                      pi_out.data_ptr(), scratch.data_ptr(), nb, stream)
        assert rec["step"] == 5
        got_phi = host(phi_out).reshape((nz + 2 * T,) + plane)
        got_pi = host(pi_out).reshape((nz + 2 * T,) + plane)
        np.testing.assert_array_equal(got_phi[T:T + nz], ref_phi[z0:z0 + nz], err_msg=str(sl))
        np.testing.assert_array_equal(got_pi[T:T + nz], ref_pi[z0:z0 + nz], err_msg=str(sl))
        links = rec["links"] if links is None else links + rec["links"]
        links_dir = rec["links_dir"] if links_dir is None else [a + b for a, b in zip(links_dir, rec["links_dir"])]
        walls += rec["wall_sites"]
        nonfinite += rec["nonfinite"]
        area += rec["area_density"] * sites
        ek += rec["gv2"] * rec["wall_sites"]
    assert links == whole["links"] and links_dir == whole["links_dir"]
    assert walls == whole["wall_sites"] and nonfinite == whole["nonfinite"] == 0
    assert walls > 0
    assert abs(area / (sites * nslab) - whole["area_density"]) <= 1e-12 * whole["area_density"]
    assert abs(ek / walls - whole["gv2"]) <= 1e-12 * whole["gv2"]


def test_slab_pass_stats_rejects_bad_scratch():
    torch = torch_mod()
    prs = gpu_prs()
    stream = prs._stream_handle(torch.cuda.current_stream())
    p2 = prs.make_params((32, 16), deta=0.2)
    bufs = [torch.zeros(32 * 20, device="cuda") for _ in range(4)]
    ptrs = [b.data_ptr() for b in bufs]
    nb = prs.prs_slab_scratch_bytes(p2, 2, (1, 8, 1))
    assert nb > 0 and prs.prs_slab_scratch_bytes(p2, 5, (1, 8, 1)) == 0
    scratch = torch.empty(nb, dtype=torch.uint8, device="cuda")
    with pytest.raises(prs.PRSError) as e:
        prs.prs_slab_pass_stats(p2, 0, 2, (1, 8, 1), *ptrs, scratch.data_ptr(), nb - 1, stream)
    assert e.value.status == prs.PRS_ENOMEM
    with pytest.raises(prs.PRSError) as e:
        prs.prs_slab_pass_stats(p2, 0, 2, (1, 8, 1), *ptrs, None, nb, stream)
    assert e.value.status == prs.PRS_EINVAL
