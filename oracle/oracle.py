"""FP64 CPU oracle for the PRS domain-wall evolution (arXiv:1710.10420, Sec. II).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark load this module; the product package never imports it
and shares no code with it.

The arithmetic lives in ``prs_oracle.c`` (plain loops, double precision,
``-ffp-contract=off``); this module builds it with gcc, marshals numpy arrays
through ctypes and adds the exponent fit of Eq. (9), which is host
post-processing:

* ``step``      one step of Eqs. (3)-(6)
* ``stats``     the diagnostics of Eqs. (7) and (8)
* ``run``       many steps with diagnostics every K steps
* ``energy``    discrete flat-space energy (invariant used by the tests)
* ``adjoint``   reverse-mode gradient of sum V(phi^S)/V0 w.r.t. phi^0,
                phi_dot^{-1/2} and W0, with store/recompute checkpoints
* ``fit_exponent``  least-squares slope in log-log, Eq. (9)
"""
import ctypes
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "prs_oracle.c")
_LIB = os.path.join(_HERE, "libprs_oracle.so")
_lock = threading.Lock()
_lib = None


class Params(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3),
        ("dx", ctypes.c_double),
        ("deta", ctypes.c_double),
        ("eta0", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("m", ctypes.c_double),
        ("V0", ctypes.c_double),
        ("W0", ctypes.c_double),
        ("phi0", ctypes.c_double),
        ("beta", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
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


def build(force=False):
    """Compile prs_oracle.c into libprs_oracle.so next to it (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            P = ctypes.POINTER(Params)
            D = ctypes.POINTER(ctypes.c_double)
            S = ctypes.POINTER(Stats)
            i64 = ctypes.c_int64
            lib.orc_step.argtypes = [P, i64, D, D, D]
            lib.orc_step.restype = None
            lib.orc_stats.argtypes = [P, i64, D, D, S]
            lib.orc_stats.restype = None
            lib.orc_run.argtypes = [P, i64, i64, ctypes.c_int32, D, D, S, i64]
            lib.orc_run.restype = i64
            lib.orc_energy.argtypes = [P, D, D, D]
            lib.orc_energy.restype = ctypes.c_double
            lib.orc_loss.argtypes = [P, D]
            lib.orc_loss.restype = ctypes.c_double
            lib.orc_adjoint.argtypes = [P, i64, i64, ctypes.c_int32, D, D, D, D, D, D]
            lib.orc_adjoint.restype = ctypes.c_int
            lib.orc_delta.argtypes = [P, i64]
            lib.orc_delta.restype = ctypes.c_double
            lib.orc_set_progress.argtypes = [ctypes.c_int]
            lib.orc_set_progress.restype = None
            _lib = lib
    return _lib


class using_library:
    """Context manager that points this module at another build of the
    oracle source (used by the mutation tests, which compile deliberately
    wrong copies and check that the pins reject them)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        _load()
        self.saved = _lib
        lib = ctypes.CDLL(self.path)
        for name in ("orc_step", "orc_stats", "orc_run", "orc_energy", "orc_loss", "orc_adjoint",
                     "orc_delta"):
            f, g = getattr(self.saved, name), getattr(lib, name)
            g.argtypes, g.restype = f.argtypes, f.restype
        _lib = lib
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def build_variant(source_text, out_path):
    """Compile a modified oracle source to out_path (test use only)."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(source_text)
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                    "-shared", "-std=c11", "-o", out_path, src, "-lm"], check=True)
    return out_path


def source_text():
    with open(_SRC) as f:
        return f.read()


def set_progress(on):
    """Print one line per segment of the adjoint's reverse sweep (stdout)."""
    _load().orc_set_progress(1 if on else 0)


def set_threads(n):
    """Set the OpenMP thread count used by the oracle's loops."""
    libgomp = ctypes.CDLL("libgomp.so.1")
    libgomp.omp_set_num_threads(int(n))


def v0_of_w0(W0):
    """V0 = pi^2 / (2 W0^2): the continuum kink tanh(pi x / W0) then solves
    (1/2) phi'^2 = V exactly (V0 and W0 are not given in the paper)."""
    return 0.0 if math.isinf(W0) else math.pi ** 2 / (2.0 * W0 * W0)


def params(shape, deta, eta0=1.0, alpha=3.0, m=1.0, W0=10.0, dx=1.0, phi0=1.0, V0=None, beta=0.0):
    """Build oracle parameters.  ``shape`` is (nx, ny) or (nx, ny, nz);
    ``beta`` is the scale-factor power of the force (0: PRS)."""
    p = Params()
    p.ndim = len(shape)
    if p.ndim not in (2, 3):
        raise ValueError("ndim must be 2 or 3")
    for d in range(3):
        p.n[d] = int(shape[d]) if d < len(shape) else 1
    p.dx, p.deta, p.eta0, p.alpha, p.m = dx, deta, eta0, alpha, m
    p.W0 = W0
    p.V0 = v0_of_w0(W0) if V0 is None else V0
    p.phi0 = phi0
    p.beta = beta
    return p


def _dptr(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _nsites(p):
    return p.n[0] * p.n[1] * (p.n[2] if p.ndim == 3 else 1)


def _field(a, p):
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    if a.size != _nsites(p):
        raise ValueError("field has %d sites, lattice has %d" % (a.size, _nsites(p)))
    return a


def step(p, n, phi, pi):
    """One step n -> n+1; returns (phi^{n+1}, phi_dot^{n+1/2}) as new arrays."""
    lib = _load()
    phi = _field(phi, p).copy()
    pi = _field(pi, p).copy()
    out = np.empty_like(phi)
    lib.orc_step(ctypes.byref(p), n, _dptr(phi), _dptr(pi), _dptr(out))
    return out, pi


def stats(p, phi, pi, n=0):
    """Diagnostics of state n as a dict."""
    lib = _load()
    phi = _field(phi, p)
    pi = _field(pi, p)
    s = Stats()
    lib.orc_stats(ctypes.byref(p), n, _dptr(phi), _dptr(pi), ctypes.byref(s))
    return s.as_dict()


def run(p, phi, pi, nsteps, n0=0, diag_every=0):
    """Advance nsteps from step n0.  Returns (phi, pi, records) where records
    holds the diagnostics of every state n0 <= n < n0+nsteps with
    n % diag_every == 0."""
    lib = _load()
    phi = _field(phi, p).copy()
    pi = _field(pi, p).copy()
    cap = 0
    if diag_every > 0:
        first = -(-n0 // diag_every) * diag_every
        cap = max(0, (n0 + nsteps - 1 - first) // diag_every + 1) if nsteps > 0 else 0
    series = (Stats * max(cap, 1))()
    k = lib.orc_run(ctypes.byref(p), n0, nsteps, diag_every, _dptr(phi), _dptr(pi),
                    series, cap)
    return phi, pi, [series[i].as_dict() for i in range(k)]


def energy(p, phi, pi_prev, pi_next):
    lib = _load()
    return lib.orc_energy(ctypes.byref(p), _dptr(_field(phi, p)), _dptr(_field(pi_prev, p)),
                          _dptr(_field(pi_next, p)))


def loss(p, phi):
    """sum over sites of V(phi)/V0."""
    return _load().orc_loss(ctypes.byref(p), _dptr(_field(phi, p)))


def delta(p, n):
    return _load().orc_delta(ctypes.byref(p), n)


def adjoint(p, phi0, pi0, nsteps, ckpt_every=64, n0=0):
    """Gradient of L = sum V(phi^S)/V0 (S = n0 + nsteps).

    Returns dict(loss, grad_phi, grad_pi, dL_dV0, grad_W0) where grad_W0 uses
    V0 = pi^2/(2 W0^2), i.e. dV0/dW0 = -2 V0 / W0."""
    lib = _load()
    phi0 = _field(phi0, p)
    pi0 = _field(pi0, p)
    gphi = np.empty_like(phi0)
    gpi = np.empty_like(phi0)
    dv0 = ctypes.c_double()
    ls = ctypes.c_double()
    rc = lib.orc_adjoint(ctypes.byref(p), n0, nsteps, ckpt_every, _dptr(phi0), _dptr(pi0),
                         _dptr(gphi), _dptr(gpi), ctypes.byref(dv0), ctypes.byref(ls))
    if rc != 0:
        raise MemoryError("oracle adjoint could not allocate its checkpoints")
    gw0 = dv0.value * (-2.0 * p.V0 / p.W0) if (p.W0 > 0 and not math.isinf(p.W0)) else 0.0
    return {"loss": ls.value, "grad_phi": gphi, "grad_pi": gpi,
            "dL_dV0": dv0.value, "grad_W0": gw0}


def fit_exponent(eta, y, eta_min=None, eta_max=None):
    """Ordinary least-squares slope of ln y against ln eta (Eq. 9), over the
    points with eta_min <= eta <= eta_max.  Unweighted, as the paper gives no
    weights."""
    eta = np.asarray(eta, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    sel = np.ones(eta.shape, dtype=bool)
    if eta_min is not None:
        sel &= eta >= eta_min
    if eta_max is not None:
        sel &= eta <= eta_max
    sel &= y > 0
    lx = np.log(eta[sel])
    ly = np.log(y[sel])
    if lx.size < 2:
        return float("nan")
    mx, my = lx.mean(), ly.mean()
    return float(((lx - mx) * (ly - my)).sum() / ((lx - mx) ** 2).sum())


def scaling_exponents(records, eta_min=None, eta_max=None):
    """(mu, nu) of Eq. (9): rho ~ eta^mu and gamma v ~ eta^nu, the latter from
    the slope of (gamma v)^2 halved."""
    eta = [r["eta"] for r in records]
    mu = fit_exponent(eta, [r["area_density"] for r in records], eta_min, eta_max)
    nu2 = fit_exponent(eta, [r["gv2"] for r in records], eta_min, eta_max)
    return mu, 0.5 * nu2
