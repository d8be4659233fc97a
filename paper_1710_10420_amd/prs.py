"""ctypes binding of libprs.so (the C ABI of include/prs.h).

Argument marshalling only: every step of the evolution runs in the library's
HIP kernels.  PyTorch supplies device memory and the current HIP stream.
Importing this module raises ImportError when libprs.so has not been built;
there is no fallback implementation.
"""
import ctypes
import math
import os

# torch carries its own HIP runtime (SONAME libamdhip64.so.7).  Loading torch
# first makes libprs.so bind to that same runtime, so device pointers and
# streams created by torch are valid in the library; loading the library first
# would pull in a second runtime from /opt/rocm.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libprs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libprs.so is not built (run python -m paper_1710_10420_amd.build); "
                      "the PRS path has no non-HIP fallback")

_lib = ctypes.CDLL(LIB_PATH)

PRS_OK = 0
PRS_EINVAL = -1
PRS_ENOMEM = -2
PRS_EDEVICE = -3
PRS_ESTATE = -4
PRS_EUNSUPPORTED = -5


class prs_params(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("diag_every", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3),
        ("dx", ctypes.c_double),
        ("deta", ctypes.c_double),
        ("eta0", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("beta", ctypes.c_double),
        ("m", ctypes.c_double),
        ("W0", ctypes.c_double),
        ("phi0", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


PRS_F32 = 0
PRS_F64 = 1


class prs_stats(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64),
        ("eta", ctypes.c_double),
        ("links", ctypes.c_uint64),
        ("links_dir", ctypes.c_uint64 * 3),
        ("wall_sites", ctypes.c_uint64),
        ("nonfinite", ctypes.c_uint64),
        ("area_density", ctypes.c_double),
        ("gv2", ctypes.c_double),
    ]

    def as_dict(self):
        return {
            "step": int(self.step),
            "eta": float(self.eta),
            "links": int(self.links),
            "links_dir": [int(v) for v in self.links_dir],
            "wall_sites": int(self.wall_sites),
            "nonfinite": int(self.nonfinite),
            "area_density": float(self.area_density),
            "gv2": float(self.gv2),
        }


class prs_batch_item(ctypes.Structure):
    _fields_ = [
        ("p", prs_params),
        ("nsteps", ctypes.c_int64),
        ("seed", ctypes.c_uint64),
        ("init_from_seed", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("phi_a", ctypes.c_void_p),
        ("phi_b", ctypes.c_void_p),
        ("dphi", ctypes.c_void_p),
    ]


PRS_BATCH_PERSISTENT_GRAPH = 0
PRS_BATCH_PERSISTENT = 1
PRS_BATCH_PER_STEP = 2
PRS_BATCH_STREAMS_GRAPH = 3
PRS_BATCH_STREAMS = 4

_P = ctypes.POINTER(prs_params)
_S = ctypes.POINTER(prs_stats)
_vp = ctypes.c_void_p
_i32, _i64, _u64, _sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
_d = ctypes.c_double


def _decl(name, restype, *argtypes):
    f = getattr(_lib, name)
    f.restype = restype
    f.argtypes = list(argtypes)
    return f


_decl("prs_workspace_bytes", _sz, _P)
_decl("prs_init", _i32, _P, _vp, _vp, _vp, _vp, _sz, _vp, ctypes.POINTER(_vp))
_decl("prs_records_in", _i64, _P, _i64, _i64)
_decl("prs_step_n", _i32, _vp, _i64, _S, _i64, ctypes.POINTER(_i64))
_decl("prs_wall_stats", _i32, _vp, _S)
_decl("prs_get_state", _i32, _vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
      ctypes.POINTER(_i64), ctypes.POINTER(_d))
_decl("prs_set_state", _i32, _vp, _vp, _vp, _i64)
_decl("prs_set_tiling", _i32, _vp, _i32, _i32, _i32)
_decl("prs_get_tiling", _i32, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32))
_decl("prs_destroy", None, _vp)
_decl("prs_fill_uniform", _i32, _vp, _i64, _u64, _vp)
_decl("prs_fill_uniform_f64", _i32, _vp, _i64, _u64, _vp)
_decl("prs_fit_scaling", _i32, _S, _i64, _d, _d, ctypes.POINTER(_d), ctypes.POINTER(_d))
_decl("prs_adjoint_workspace_bytes", _sz, _P, _i64, _i32)
_decl("prs_adjoint_forward", _i32, _vp, _i64, _i32, _vp, _sz, ctypes.POINTER(_d))
_decl("prs_adjoint_backward", _i32, _vp, _vp, _sz, _vp, _vp, ctypes.POINTER(_d))
_decl("prs_adjoint", _i32, _vp, _i64, _i32, _vp, _sz, _vp, _vp, ctypes.POINTER(_d), ctypes.POINTER(_d))
_BI = ctypes.POINTER(prs_batch_item)
_decl("prs_batch_workspace_bytes", _sz, _BI, _i32)
_decl("prs_batch_create", _i32, _BI, _i32, _vp, _sz, _vp, ctypes.POINTER(_vp))
_decl("prs_batch_offsets", _i32, _vp, ctypes.POINTER(_i64))
_decl("prs_batch_set_tiling", _i32, _vp, _i32, _i32, _i32, _i32)
_decl("prs_batch_set_mode", _i32, _vp, _i32)
_decl("prs_batch_set_time_blocking", _i32, _vp, _i32, _i32)
_decl("prs_batch_state", _i32, _vp, _i32, ctypes.POINTER(_vp), ctypes.POINTER(_vp))
_decl("prs_batch_run", _i32, _vp, _S, _i64)
_decl("prs_batch_autotune", _i32, _vp, ctypes.POINTER(_d))
_decl("prs_batch_get_tiling", _i32, _vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32),
      ctypes.POINTER(_i32))
_decl("prs_batch_destroy", None, _vp)
_decl("prs_autotune", _i32, _vp, ctypes.c_char_p, _i32, _vp, _sz, ctypes.POINTER(_d))
_decl("prs_tune_workspace_bytes", _sz, _vp, _i32)
_decl("prs_set_launch_timing", _i32, _vp, _i32)
_decl("prs_get_launch_timing", _i32, _vp, ctypes.POINTER(_d), ctypes.POINTER(_i64), _i32)
_decl("prs_copy", _i32, _vp, _vp, _sz, _vp)
_decl("prs_set_adjoint_scheme", _i32, _vp, _i32)
_decl("prs_slab_pass_stats_static", _i32, _P, _i64, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp)
_decl("prs_get_adjoint_scheme", _i32, _vp, ctypes.POINTER(_i32))
_decl("prs_tuned_tiling", _i32, _P, ctypes.c_char_p, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
      ctypes.POINTER(_i32))
_decl("prs_set_time_blocking", _i32, _vp, _i32)
_decl("prs_set_adjoint_tiling", _i32, _vp, _i32, _i32, _i32)
_decl("prs_plan_passes", _i32, _vp, _i64, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i64))
_decl("prs_get_adjoint_tiling", _i32, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32))
_decl("prs_get_time_blocking", _i32, _vp, ctypes.POINTER(_i32))
_decl("prs_set_adjoint_time_blocking", _i32, _vp, _i32)
_decl("prs_get_adjoint_time_blocking", _i32, _vp, ctypes.POINTER(_i32))
_decl("prs_set_recompute_tiling", _i32, _vp, _i32, _i32, _i32, _i32)
_decl("prs_slab_pass", _i32, _P, _i64, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp)
_decl("prs_slab_pass_stats", _i32, _P, _i64, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _sz, _S, _vp)
_decl("prs_slab_scratch_bytes", _sz, _P, _i32, _i32, _i32, _i32)
_decl("prs_get_recompute_tiling", _i32, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32),
      ctypes.POINTER(_i32))
_decl("prs_strerror", ctypes.c_char_p, _i32)
_decl("prs_last_error", ctypes.c_char_p)

EXPORTED = [
    "prs_workspace_bytes", "prs_init", "prs_records_in", "prs_step_n", "prs_wall_stats",
    "prs_get_state", "prs_set_state", "prs_set_tiling", "prs_get_tiling", "prs_destroy",
    "prs_fill_uniform", "prs_fit_scaling", "prs_strerror", "prs_last_error",
    "prs_adjoint_workspace_bytes", "prs_adjoint_forward", "prs_adjoint_backward", "prs_adjoint",
    "prs_batch_workspace_bytes", "prs_batch_create", "prs_batch_offsets", "prs_batch_set_tiling",
    "prs_batch_set_mode", "prs_batch_run", "prs_batch_destroy", "prs_batch_set_time_blocking",
    "prs_batch_state", "prs_batch_autotune", "prs_batch_get_tiling", "prs_autotune", "prs_tuned_tiling",
    "prs_set_time_blocking", "prs_get_time_blocking", "prs_set_adjoint_tiling",
    "prs_get_adjoint_tiling", "prs_plan_passes", "prs_fill_uniform_f64",
    "prs_set_adjoint_time_blocking", "prs_get_adjoint_time_blocking",
    "prs_set_recompute_tiling", "prs_get_recompute_tiling", "prs_slab_pass",
    "prs_slab_pass_stats", "prs_slab_scratch_bytes", "prs_tune_workspace_bytes",
    "prs_set_launch_timing", "prs_get_launch_timing", "prs_copy", "prs_set_adjoint_scheme",
    "prs_get_adjoint_scheme", "prs_slab_pass_stats_static",
]

PRS_TUNE_FORCE = 1
PRS_TUNE_BATCH = 2
PRS_TUNE_ADJOINT = 4
PRS_TUNE_MIN_WORKSPACE = 8
PRS_ADJ_STORED = 0
PRS_ADJ_FUSED = 1


class PRSError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.prs_last_error().decode() or _lib.prs_strerror(status).decode()
        super().__init__("%s failed (%d, %s): %s" % (where, status,
                                                     _lib.prs_strerror(status).decode(), msg))


def _check(status, where):
    if status != PRS_OK:
        raise PRSError(status, where)


def make_params(shape, deta, eta0=1.0, alpha=3.0, m=1.0, W0=10.0, dx=1.0, phi0=1.0,
                beta=0.0, diag_every=0, precision=PRS_F32):
    """prs_params for a lattice of shape (nx, ny) or (nx, ny, nz); precision
    PRS_F32 (float32 fields) or PRS_F64 (float64 fields)."""
    p = prs_params()
    p.precision = int(precision)
    p.ndim = len(shape)
    for d in range(3):
        p.n[d] = int(shape[d]) if d < len(shape) else 1
    p.dx, p.deta, p.eta0, p.alpha, p.beta, p.m = dx, deta, eta0, alpha, beta, m
    p.W0, p.phi0 = W0, phi0
    p.diag_every = int(diag_every)
    return p


def sites(p):
    return p.n[0] * p.n[1] * (p.n[2] if p.ndim == 3 else 1)


def field_dtype(p):
    """torch dtype of the fields of a run with parameters p."""
    return torch.float64 if p.precision == PRS_F64 else torch.float32


def _stream_handle(stream):
    return ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)


# ---- thin wrappers with the C names -----------------------------------

def prs_workspace_bytes(p):
    return int(_lib.prs_workspace_bytes(ctypes.byref(p)))


def prs_records_in(p, n0, nsteps):
    return int(_lib.prs_records_in(ctypes.byref(p), n0, nsteps))


def prs_init(p, phi_a, phi_b, dphi, workspace, ws_bytes, stream):
    ctx = ctypes.c_void_p()
    _check(_lib.prs_init(ctypes.byref(p), phi_a, phi_b, dphi, workspace, ws_bytes,
                         stream, ctypes.byref(ctx)), "prs_init")
    return ctx


def prs_step_n(ctx, nsteps, cap):
    """Returns the list of records (empty when cap == 0)."""
    series = (prs_stats * max(cap, 1))() if cap > 0 else None
    nw = _i64(0)
    _check(_lib.prs_step_n(ctx, nsteps, series, cap, ctypes.byref(nw)), "prs_step_n")
    return [series[i].as_dict() for i in range(nw.value)] if series is not None else []


def prs_wall_stats(ctx):
    s = prs_stats()
    _check(_lib.prs_wall_stats(ctx, ctypes.byref(s)), "prs_wall_stats")
    return s.as_dict()


def prs_get_state(ctx):
    phi, dphi, step, eta = _vp(), _vp(), _i64(), _d()
    _check(_lib.prs_get_state(ctx, ctypes.byref(phi), ctypes.byref(dphi), ctypes.byref(step),
                              ctypes.byref(eta)), "prs_get_state")
    return phi.value, dphi.value, step.value, eta.value


def prs_set_state(ctx, phi, dphi, step):
    _check(_lib.prs_set_state(ctx, phi, dphi, step), "prs_set_state")


def prs_set_tiling(ctx, vec, rows, ty=1):
    _check(_lib.prs_set_tiling(ctx, vec, rows, ty), "prs_set_tiling")


def prs_get_tiling(ctx):
    v, r, t = _i32(), _i32(), _i32()
    _check(_lib.prs_get_tiling(ctx, ctypes.byref(v), ctypes.byref(r), ctypes.byref(t)),
           "prs_get_tiling")
    return v.value, r.value, t.value


def prs_set_time_blocking(ctx, steps_per_pass):
    _check(_lib.prs_set_time_blocking(ctx, steps_per_pass), "prs_set_time_blocking")


def prs_get_time_blocking(ctx):
    v = _i32()
    _check(_lib.prs_get_time_blocking(ctx, ctypes.byref(v)), "prs_get_time_blocking")
    return v.value


def prs_set_adjoint_tiling(ctx, vec, rows, ty=1):
    _check(_lib.prs_set_adjoint_tiling(ctx, vec, rows, ty), "prs_set_adjoint_tiling")


def prs_get_adjoint_tiling(ctx):
    v, r, t = _i32(), _i32(), _i32()
    _check(_lib.prs_get_adjoint_tiling(ctx, ctypes.byref(v), ctypes.byref(r), ctypes.byref(t)),
           "prs_get_adjoint_tiling")
    return v.value, r.value, t.value


def prs_set_adjoint_time_blocking(ctx, steps_per_pass):
    _check(_lib.prs_set_adjoint_time_blocking(ctx, steps_per_pass), "prs_set_adjoint_time_blocking")


def prs_get_adjoint_time_blocking(ctx):
    v = _i32()
    _check(_lib.prs_get_adjoint_time_blocking(ctx, ctypes.byref(v)), "prs_get_adjoint_time_blocking")
    return v.value


def prs_set_recompute_tiling(ctx, vec, rows, ty, steps_per_pass):
    _check(_lib.prs_set_recompute_tiling(ctx, vec, rows, ty, steps_per_pass), "prs_set_recompute_tiling")


def prs_get_recompute_tiling(ctx):
    """(vec, rows, ty, steps per pass) of the adjoint's recomputation."""
    v = [_i32() for _ in range(4)]
    _check(_lib.prs_get_recompute_tiling(ctx, *(ctypes.byref(x) for x in v)), "prs_get_recompute_tiling")
    return tuple(x.value for x in v)


def prs_slab_pass(p, n0, steps, tiling, phi_in, phi_out, pi_in, pi_out, stream):
    """One multi-step pass over a slab of a lattice cut along its last axis
    (y in 2D, z in 3D), stored with `steps` halo rows or planes below and
    above (device pointers; see include/prs.h)."""
    _check(_lib.prs_slab_pass(ctypes.byref(p), n0, steps, tiling[0], tiling[1], tiling[2], phi_in, phi_out,
                              pi_in, pi_out, stream), "prs_slab_pass")


def prs_slab_scratch_bytes(p, steps, tiling):
    """Scratch bytes prs_slab_pass_stats needs (0: no such pass)."""
    return int(_lib.prs_slab_scratch_bytes(ctypes.byref(p), steps, tiling[0], tiling[1], tiling[2]))


def prs_slab_pass_stats(p, n0, steps, tiling, phi_in, phi_out, pi_in, pi_out, scratch, scratch_bytes, stream):
    """prs_slab_pass with the input state's wall diagnostics over the slab's
    interior; returns the record as a dict (synchronises the stream)."""
    rec = prs_stats()
    _check(_lib.prs_slab_pass_stats(ctypes.byref(p), n0, steps, tiling[0], tiling[1], tiling[2], phi_in, phi_out,
                                    pi_in, pi_out, scratch, scratch_bytes, ctypes.byref(rec), stream),
           "prs_slab_pass_stats")
    return rec.as_dict()


def prs_slab_pass_stats_static(p, n0, steps, tiling, phi_in, phi_out, pi_in, pi_out, record_dev, stream):
    """prs_slab_pass_stats without any allocation: the library's static
    scratch, the record written to the device pointer record_dev (one
    prs_stats, no synchronisation)."""
    _check(_lib.prs_slab_pass_stats_static(ctypes.byref(p), n0, steps, tiling[0], tiling[1], tiling[2], phi_in,
                                           phi_out, pi_in, pi_out, record_dev, stream),
           "prs_slab_pass_stats_static")


def prs_stats_from_bytes(raw):
    """A prs_stats record (as a dict) from its bytes, e.g. a device record
    copied to the host."""
    rec = prs_stats.from_buffer_copy(bytes(raw))
    return rec.as_dict()


def prs_plan_passes(ctx, nsteps, with_records=True):
    """(multi-step passes, single-step passes) prs_step_n would launch."""
    m, n1 = _i64(), _i64()
    _check(_lib.prs_plan_passes(ctx, nsteps, 1 if with_records else 0, ctypes.byref(m), ctypes.byref(n1)),
           "prs_plan_passes")
    return m.value, n1.value


def prs_destroy(ctx):
    _lib.prs_destroy(ctx)


def prs_fill_uniform(phi_ptr, count, seed, stream):
    _check(_lib.prs_fill_uniform(phi_ptr, count, seed, stream), "prs_fill_uniform")


def prs_fill_uniform_f64(phi_ptr, count, seed, stream):
    _check(_lib.prs_fill_uniform_f64(phi_ptr, count, seed, stream), "prs_fill_uniform_f64")


def prs_fit_scaling(records, eta_min=0.0, eta_max=math.inf):
    arr = (prs_stats * max(len(records), 1))()
    for i, r in enumerate(records):
        s = arr[i]
        s.step, s.eta = r["step"], r["eta"]
        s.links, s.wall_sites, s.nonfinite = r["links"], r["wall_sites"], r["nonfinite"]
        for d in range(3):
            s.links_dir[d] = r["links_dir"][d]
        s.area_density, s.gv2 = r["area_density"], r["gv2"]
    mu, nu = _d(), _d()
    _check(_lib.prs_fit_scaling(arr, len(records), eta_min, eta_max, ctypes.byref(mu),
                                ctypes.byref(nu)), "prs_fit_scaling")
    return mu.value, nu.value


def prs_adjoint_workspace_bytes(p, nsteps, ckpt_every):
    return int(_lib.prs_adjoint_workspace_bytes(ctypes.byref(p), nsteps, ckpt_every))


def prs_adjoint_forward(ctx, nsteps, ckpt_every, work, work_bytes):
    loss = _d()
    _check(_lib.prs_adjoint_forward(ctx, nsteps, ckpt_every, work, work_bytes, ctypes.byref(loss)),
           "prs_adjoint_forward")
    return loss.value


def prs_adjoint_backward(ctx, work, work_bytes, grad_phi0, grad_dphi0):
    gw = _d()
    _check(_lib.prs_adjoint_backward(ctx, work, work_bytes, grad_phi0, grad_dphi0, ctypes.byref(gw)),
           "prs_adjoint_backward")
    return gw.value


def prs_adjoint(ctx, nsteps, ckpt_every, work, work_bytes, grad_phi0, grad_dphi0):
    gw, loss = _d(), _d()
    _check(_lib.prs_adjoint(ctx, nsteps, ckpt_every, work, work_bytes, grad_phi0, grad_dphi0,
                            ctypes.byref(gw), ctypes.byref(loss)), "prs_adjoint")
    return loss.value, gw.value


def prs_batch_workspace_bytes(items):
    arr = (prs_batch_item * len(items))(*items)
    return int(_lib.prs_batch_workspace_bytes(arr, len(items)))


def prs_batch_create(items, workspace, ws_bytes, stream):
    arr = (prs_batch_item * len(items))(*items)
    b = ctypes.c_void_p()
    _check(_lib.prs_batch_create(arr, len(items), workspace, ws_bytes, stream, ctypes.byref(b)),
           "prs_batch_create")
    return b


def prs_batch_offsets(b, count):
    off = (_i64 * (count + 1))()
    _check(_lib.prs_batch_offsets(b, off), "prs_batch_offsets")
    return [int(v) for v in off]


def prs_batch_set_tiling(b, item, vec, rows, ty=1):
    _check(_lib.prs_batch_set_tiling(b, item, vec, rows, ty), "prs_batch_set_tiling")


def prs_batch_set_mode(b, mode):
    _check(_lib.prs_batch_set_mode(b, mode), "prs_batch_set_mode")


def prs_batch_set_time_blocking(b, item, steps_per_pass):
    _check(_lib.prs_batch_set_time_blocking(b, item, steps_per_pass), "prs_batch_set_time_blocking")


def prs_batch_state(b, item):
    phi, dphi = _vp(), _vp()
    _check(_lib.prs_batch_state(b, item, ctypes.byref(phi), ctypes.byref(dphi)), "prs_batch_state")
    return phi.value, dphi.value


def prs_batch_run(b, total_records):
    series = (prs_stats * max(total_records, 1))()
    _check(_lib.prs_batch_run(b, series, total_records), "prs_batch_run")
    return [series[i].as_dict() for i in range(total_records)]


def prs_batch_autotune(b):
    """Time of one ensemble run (ms) with the settings the tuner kept."""
    ms = _d()
    _check(_lib.prs_batch_autotune(b, ctypes.byref(ms)), "prs_batch_autotune")
    return ms.value


def prs_batch_get_tiling(b, item):
    """((vec, rows, ty), steps_per_pass) of one item."""
    v = [_i32() for _ in range(4)]
    _check(_lib.prs_batch_get_tiling(b, item, *(ctypes.byref(x) for x in v)), "prs_batch_get_tiling")
    return (v[0].value, v[1].value, v[2].value), v[3].value


def prs_batch_destroy(b):
    _lib.prs_batch_destroy(b)


def prs_tune_workspace_bytes(ctx, flags=0):
    return int(_lib.prs_tune_workspace_bytes(ctx, flags))


def prs_autotune(ctx, cache_path=None, flags=0, work=None):
    """Returns the time of one step (us) with the chosen tiling.  `work` is
    a device tensor of scratch (the tuner allocates nothing); by default one
    of prs_tune_workspace_bytes(ctx, flags) bytes is allocated here, or, for
    the adjoint tuner when that does not fit, of the least size it takes."""
    us = _d()
    path = cache_path.encode() if cache_path else None
    if work is None:
        try:
            work = torch.empty(prs_tune_workspace_bytes(ctx, flags), dtype=torch.uint8, device="cuda")
        except torch.OutOfMemoryError:
            if not flags & PRS_TUNE_ADJOINT:
                raise
            torch.cuda.empty_cache()
            work = torch.empty(prs_tune_workspace_bytes(ctx, flags | PRS_TUNE_MIN_WORKSPACE),
                               dtype=torch.uint8, device="cuda")
    _check(_lib.prs_autotune(ctx, path, flags, work.data_ptr(), work.numel() * work.element_size(),
                             ctypes.byref(us)), "prs_autotune")
    del work
    return us.value


def prs_set_launch_timing(ctx, on):
    _check(_lib.prs_set_launch_timing(ctx, 1 if on else 0), "prs_set_launch_timing")


def prs_get_launch_timing(ctx, reset=True):
    """(total milliseconds, launches) of the pass kernel since the last reset."""
    ms, n = _d(), _i64()
    _check(_lib.prs_get_launch_timing(ctx, ctypes.byref(ms), ctypes.byref(n), 1 if reset else 0),
           "prs_get_launch_timing")
    return ms.value, n.value


def prs_set_adjoint_scheme(ctx, scheme):
    _check(_lib.prs_set_adjoint_scheme(ctx, scheme), "prs_set_adjoint_scheme")


def prs_get_adjoint_scheme(ctx):
    v = _i32()
    _check(_lib.prs_get_adjoint_scheme(ctx, ctypes.byref(v)), "prs_get_adjoint_scheme")
    return v.value


def prs_copy(dst, src, nbytes, stream):
    _check(_lib.prs_copy(dst, src, nbytes, stream), "prs_copy")


def prs_tuned_tiling(p, cache_path, flags=0):
    """Cached (vec, rows, ty) or None."""
    v, r, t = _i32(), _i32(), _i32()
    st = _lib.prs_tuned_tiling(ctypes.byref(p), cache_path.encode(), flags, ctypes.byref(v),
                               ctypes.byref(r), ctypes.byref(t))
    if st == PRS_ESTATE:
        return None
    _check(st, "prs_tuned_tiling")
    return v.value, r.value, t.value


# ---- convenience object over torch-owned buffers ----------------------

class Sim:
    """One PRS run on the current CUDA (HIP) device.

    phi0: a tensor with the initial field in site order (any shape with the
    right number of elements; converted to the run's precision), or None to
    draw it with prs_fill_uniform(seed).  dphi0: initial phi_dot^{-1/2}
    (default 0).  Fields are float32, or float64 when p.precision is
    PRS_F64."""

    def __init__(self, p, phi0=None, dphi0=None, seed=1, device="cuda", stream=None):
        import torch
        self.torch = torch
        self.p = p
        n = sites(p)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self._s = _stream_handle(self.stream)
        self.dtype = field_dtype(p)
        with torch.cuda.stream(self.stream):
            self.phi_a = torch.empty(n, dtype=self.dtype, device=device)
            self.phi_b = torch.empty(n, dtype=self.dtype, device=device)
            self.dphi = torch.zeros(n, dtype=self.dtype, device=device)
            ws = prs_workspace_bytes(p)
            if ws == 0:
                raise PRSError(PRS_EINVAL, "prs_workspace_bytes")
            self.ws = torch.empty(ws, dtype=torch.uint8, device=device)
            if phi0 is None:
                fill = prs_fill_uniform_f64 if p.precision == PRS_F64 else prs_fill_uniform
                fill(self.phi_a.data_ptr(), n, seed, self._s)
            else:
                self.phi_a.copy_(phi0.reshape(-1).to(device=device, dtype=self.dtype))
            if dphi0 is not None:
                self.dphi.copy_(dphi0.reshape(-1).to(device=device, dtype=self.dtype))
        self.ctx = prs_init(p, self.phi_a.data_ptr(), self.phi_b.data_ptr(), self.dphi.data_ptr(),
                            self.ws.data_ptr(), self.ws.numel(), self._s)

    def close(self):
        if self.ctx is not None:
            prs_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def step(self):
        return prs_get_state(self.ctx)[2]

    def step_n(self, nsteps, diag=True):
        cap = prs_records_in(self.p, self.step, nsteps) if diag and self.p.diag_every > 0 else 0
        return prs_step_n(self.ctx, nsteps, cap)

    def wall_stats(self):
        return prs_wall_stats(self.ctx)

    def state(self):
        """(phi, dphi) tensors of the current state (views of the buffers)."""
        phi_ptr, _, _, _ = prs_get_state(self.ctx)
        phi = self.phi_a if phi_ptr == self.phi_a.data_ptr() else self.phi_b
        return phi, self.dphi

    def set_state(self, phi, dphi, step):
        with self.torch.cuda.stream(self.stream):
            phi = phi.reshape(-1).to(device=self.phi_a.device, dtype=self.dtype).contiguous()
            dphi = dphi.reshape(-1).to(device=self.phi_a.device, dtype=self.dtype).contiguous()
            prs_set_state(self.ctx, phi.data_ptr(), dphi.data_ptr(), step)
            self.stream.synchronize()

    def set_tiling(self, vec, rows, ty=1):
        prs_set_tiling(self.ctx, vec, rows, ty)

    def tiling(self):
        return prs_get_tiling(self.ctx)

    def set_time_blocking(self, steps_per_pass):
        prs_set_time_blocking(self.ctx, steps_per_pass)

    def time_blocking(self):
        return prs_get_time_blocking(self.ctx)


class PRSLoss(torch.autograd.Function):
    """loss = sum_i V(phi_i^S)/V0 after `nsteps` PRS steps from (phi0, dphi0 = 0).

    forward runs the evolution on the GPU with checkpoints every
    `ckpt_every` steps (prs_adjoint_forward); backward runs the hand-written
    reverse sweep (prs_adjoint_backward) and returns dL/dphi0 and dL/dW0.

        loss = PRSLoss.apply(phi0, W0, params, nsteps, ckpt_every)

    phi0: CUDA tensor of the lattice's site count, float32 or float64 (the
    run uses the precision of phi0, whatever params.precision says); W0: 0-d
    tensor (its value replaces params.W0); params: prs_params (W0 and
    precision fields ignored).  With float64 the whole evolution and the
    reverse sweep run in double precision, which torch.autograd.gradcheck
    can check against finite differences of the same GPU code."""

    @staticmethod
    def _run_forward(p, phi0, nsteps, ckpt_every):
        sim = Sim(p, phi0=phi0, device=phi0.device)
        nbytes = prs_adjoint_workspace_bytes(p, nsteps, ckpt_every)
        if nbytes == 0:
            raise PRSError(PRS_EINVAL, "prs_adjoint_workspace_bytes")
        work = torch.empty(nbytes, dtype=torch.uint8, device=phi0.device)
        loss = prs_adjoint_forward(sim.ctx, nsteps, ckpt_every, work.data_ptr(), nbytes)
        return sim, work, nbytes, loss

    @staticmethod
    def forward(ctx, phi0, W0, params, nsteps, ckpt_every=64):
        p = prs_params()
        ctypes.pointer(p)[0] = params
        p.W0 = float(W0)
        p.precision = PRS_F64 if phi0.dtype == torch.float64 else PRS_F32
        sim, work, nbytes, loss = PRSLoss._run_forward(p, phi0.detach(), nsteps, ckpt_every)
        ctx.sim, ctx.work, ctx.nbytes = sim, work, nbytes
        ctx.p, ctx.phi0, ctx.nsteps, ctx.ckpt_every = p, phi0.detach(), nsteps, ckpt_every
        ctx.W0_dtype, ctx.W0_device = W0.dtype, W0.device
        ctx.phi_dtype = phi0.dtype
        return torch.tensor(loss, dtype=torch.float64, device=phi0.device)

    @staticmethod
    def backward(ctx, grad_out):
        if ctx.sim is None:      # a second backward over the same graph: replay the forward
            ctx.sim, ctx.work, ctx.nbytes, _ = PRSLoss._run_forward(ctx.p, ctx.phi0, ctx.nsteps,
                                                                    ctx.ckpt_every)
        sim = ctx.sim
        gphi = torch.empty_like(sim.phi_a)
        with torch.cuda.stream(sim.stream):
            gw0 = prs_adjoint_backward(sim.ctx, ctx.work.data_ptr(), ctx.nbytes, gphi.data_ptr(), None)
        sim.close()
        ctx.sim = None
        ctx.work = None
        g = grad_out.to(torch.float64)
        grad_phi = (gphi.to(torch.float64) * g).to(ctx.phi_dtype)
        grad_w0 = (g * gw0).to(dtype=ctx.W0_dtype, device=ctx.W0_device)
        return grad_phi, grad_w0, None, None, None


class Batch:
    """An ensemble of realisations run by prs_batch_run.

    specs: list of dicts with keys shape, deta, nsteps and optionally m, W0,
    alpha, beta, dx, eta0, diag_every, seed (the initial field is drawn from
    the seed at every run, dphi = 0) and precision (PRS_F32 or PRS_F64;
    float64 items run in the stream modes)."""

    def __init__(self, specs, device="cuda", stream=None):
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self._s = _stream_handle(self.stream)
        self.specs = specs
        self.items = []
        self.fields = []
        with torch.cuda.stream(self.stream):
            for sp in specs:
                p = make_params(sp["shape"], deta=sp["deta"], m=sp.get("m", 1.0), W0=sp.get("W0", 10.0),
                                alpha=sp.get("alpha", 3.0), beta=sp.get("beta", 0.0), dx=sp.get("dx", 1.0),
                                eta0=sp.get("eta0", 1.0), diag_every=sp.get("diag_every", 0),
                                precision=sp.get("precision", PRS_F32))
                n = sites(p)
                f = [torch.empty(n, dtype=field_dtype(p), device=device) for _ in range(3)]
                it = prs_batch_item()
                it.p = p
                it.nsteps = int(sp["nsteps"])
                it.seed = int(sp.get("seed", 1))
                it.init_from_seed = 1
                it.phi_a, it.phi_b, it.dphi = f[0].data_ptr(), f[1].data_ptr(), f[2].data_ptr()
                self.items.append(it)
                self.fields.append(f)
            nb = prs_batch_workspace_bytes(self.items)
            if nb == 0:
                raise PRSError(PRS_EINVAL, "prs_batch_workspace_bytes")
            self.ws = torch.empty(nb, dtype=torch.uint8, device=device)
        self.b = prs_batch_create(self.items, self.ws.data_ptr(), nb, self._s)
        self.offsets = prs_batch_offsets(self.b, len(self.items))

    def set_tiling(self, item, vec, rows, ty=1):
        prs_batch_set_tiling(self.b, item, vec, rows, ty)

    def set_mode(self, mode):
        prs_batch_set_mode(self.b, mode)

    def set_time_blocking(self, item, steps_per_pass):
        prs_batch_set_time_blocking(self.b, item, steps_per_pass)

    def tiling(self, item):
        """((vec, rows, ty), steps_per_pass) of one realisation."""
        return prs_batch_get_tiling(self.b, item)

    def autotune(self):
        """Refines the marching-tile lengths by timing the whole ensemble in
        the current mode; returns the time of one run (ms)."""
        return prs_batch_autotune(self.b)

    def run(self):
        """Runs the ensemble; returns one record list per realisation."""
        recs = prs_batch_run(self.b, self.offsets[-1])
        return [recs[self.offsets[r]:self.offsets[r + 1]] for r in range(len(self.items))]

    def final_state(self, r):
        """(phi, dphi) tensors of realisation r after its last step."""
        f = self.fields[r]
        phi_ptr, _ = prs_batch_state(self.b, r)
        return (f[0] if phi_ptr == f[0].data_ptr() else f[1]), f[2]

    def close(self):
        if self.b is not None:
            prs_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
