"""The allocation-free slab-diagnostics entry point (prs_slab_pass_stats_static)
against prs_slab_pass_stats, the entry point it varies: same pass, same
scratch layout in the library's static array instead of a caller buffer, so
fields and records must be bit for bit equal; two calls in a row, the second
on a smaller slab, and the size limit enforced before any launch."""
import ctypes

import numpy as np
import pytest

from tests.gpu_util import gpu_prs, host, say, torch_mod

pytestmark = pytest.mark.gpu


def slab_inputs(prs, torch, shape, T, seed):
    """A slab of `shape` (last axis the interior) stored with T halo planes
    per face: a seeded field and a nonzero phi_dot."""
    n = int(np.prod(shape[:-1])) * (shape[-1] + 2 * T)
    phi = torch.empty(n, dtype=torch.float32, device="cuda")
    stream = prs._stream_handle(torch.cuda.current_stream())
    prs.prs_fill_uniform(phi.data_ptr(), n, seed, stream)
    pi = torch.empty_like(phi)
    prs.prs_fill_uniform(pi.data_ptr(), n, seed + 1, stream)
    pi.mul_(0.25)
    return phi, pi, stream


def run_both(shape, T, tiling, n0, seed):
    torch = torch_mod()
    prs = gpu_prs()
    p = prs.make_params(shape, deta=0.2, m=1.0, W0=8.0)
    phi, pi, stream = slab_inputs(prs, torch, shape, T, seed)
    nb = prs.prs_slab_scratch_bytes(p, T, tiling)
    assert 0 < nb <= 4 << 20
    scratch = torch.empty(nb, dtype=torch.uint8, device="cuda")
    a_phi, a_pi = torch.zeros_like(phi), torch.zeros_like(pi)
    ref = prs.prs_slab_pass_stats(p, n0, T, tiling, phi.data_ptr(), a_phi.data_ptr(), pi.data_ptr(),
                                  a_pi.data_ptr(), scratch.data_ptr(), nb, stream)
    b_phi, b_pi = torch.zeros_like(phi), torch.zeros_like(pi)
    rec_dev = torch.zeros(ctypes.sizeof(prs.prs_stats), dtype=torch.uint8, device="cuda")
    prs.prs_slab_pass_stats_static(p, n0, T, tiling, phi.data_ptr(), b_phi.data_ptr(), pi.data_ptr(),
                                   b_pi.data_ptr(), rec_dev.data_ptr(), stream)
    torch.cuda.synchronize()
    got = prs.prs_stats_from_bytes(rec_dev.cpu().numpy().tobytes())
    np.testing.assert_array_equal(host(b_phi), host(a_phi))
    np.testing.assert_array_equal(host(b_pi), host(a_pi))
    assert got == ref, (got, ref)
    assert ref["links"] > 0 and ref["wall_sites"] > 0
    return got


def test_static_scratch_matches_caller_scratch_twice():
    say("no-alloc slab stats: 3D then a smaller 2D slab")
    big = run_both((96, 80, 40), 3, (1, 8, 2), 7, 21)
    small = run_both((64, 24), 4, (2, 8, 1), 3, 22)
    assert big["step"] == 7 and small["step"] == 3


def test_static_scratch_rejects_passes_beyond_its_size():
    """A pass whose partials exceed the 4 MiB array is refused before any
    launch (PRS_ENOMEM); the output buffers stay untouched."""
    torch = torch_mod()
    prs = gpu_prs()
    p = prs.make_params((8192, 8192), deta=0.25, m=1.0, W0=10.0)
    assert prs.prs_slab_scratch_bytes(p, 2, (1, 8, 1)) > 4 << 20
    buf = torch.zeros(1024, dtype=torch.float32, device="cuda")
    rec_dev = torch.zeros(128, dtype=torch.uint8, device="cuda")
    stream = prs._stream_handle(torch.cuda.current_stream())
    with pytest.raises(prs.PRSError) as e:
        prs.prs_slab_pass_stats_static(p, 0, 2, (1, 8, 1), buf.data_ptr(), buf.data_ptr() + 1024,
                                       buf.data_ptr() + 2048, buf.data_ptr() + 3072, rec_dev.data_ptr(), stream)
    assert e.value.status == prs.PRS_ENOMEM
    torch.cuda.synchronize()
    assert int(rec_dev.sum()) == 0 and float(buf.abs().sum()) == 0.0
