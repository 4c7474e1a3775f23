"""ctypes front end of the FP64 C oracle (``sobrc_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline of the benchmark.  The product package never imports this module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sobrc_oracle.c")
LIB = os.path.join(HERE, "libsobrc_oracle.so")

PC, PS = 0, 1
GAUSS, POISSON = 0, 1
MODE_SOBOLEV, MODE_L2, MODE_AUTO = 0, 1, 2
NEIGH_BRUTE, NEIGH_CELLS = 0, 1
TOPO_OFF, TOPO_SIMPLE = 0, 1


class Params(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("model", C.c_int32), ("ps_radius", C.c_int32),
        ("E", C.c_double), ("eps", C.c_double), ("lam", C.c_double),
        ("max_labels", C.c_int32), ("threads", C.c_int32), ("noise", C.c_int32),
        ("topo", C.c_int32), ("psf_sigma", C.c_double),
    ]


class Auto(C.Structure):
    _fields_ = [("t", C.c_int32), ("grad", C.c_int32), ("osc_prev", C.c_int32),
                ("cycle_prev", C.c_int32), ("switch_iter", C.c_int32)]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
                               "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = C.CDLL(LIB)
        P = C.POINTER
        L.ora_kernel.restype = C.c_double
        L.ora_kernel.argtypes = [C.c_double, C.c_double, C.c_double]
        L.ora_particles.restype = C.c_int64
        L.ora_particles.argtypes = [P(Params), C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
        L.ora_region_stats.restype = None
        L.ora_region_stats.argtypes = [P(Params), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.ora_l2diff.restype = None
        L.ora_l2diff.argtypes = [P(Params), C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p]
        L.ora_sobolev.restype = None
        L.ora_sobolev.argtypes = [P(Params), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_int32, C.c_int64, C.c_void_p]
        L.ora_step.restype = C.c_int64
        L.ora_step.argtypes = [P(Params), C.c_void_p, C.c_void_p, C.c_int32, C.c_int64,
                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p]
        L.ora_run.restype = C.c_int32
        L.ora_run.argtypes = [P(Params), C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                              C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.ora_auto_init.restype = None
        L.ora_auto_init.argtypes = [P(Auto), C.c_int32]
        L.ora_auto_update.restype = C.c_int32
        L.ora_auto_update.argtypes = [P(Auto), C.c_int32, C.c_double, C.c_int64, C.c_int64, C.c_int64]
        L.ora_reversals.restype = C.c_int64
        L.ora_reversals.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]
        L.ora_simple.restype = C.c_int32
        L.ora_simple.argtypes = [P(Params), C.c_void_p, C.c_int64, C.c_int32]
        L.ora_accept_ranked.restype = C.c_int64
        L.ora_accept_ranked.argtypes = [P(Params), C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]
        L.ora_psf_radius.restype = C.c_int32
        L.ora_psf_radius.argtypes = [C.c_double]
        L.ora_psf_taps.restype = None
        L.ora_psf_taps.argtypes = [C.c_double, C.c_void_p]
        L.ora_deconv_theta.restype = None
        L.ora_deconv_theta.argtypes = [P(Params), C.c_void_p, C.c_void_p, C.c_void_p]
        L.ora_deconv_model.restype = None
        L.ora_deconv_model.argtypes = [P(Params), C.c_void_p, C.c_void_p, C.c_void_p]
        L.ora_energy_pc.restype = C.c_double
        L.ora_energy_pc.argtypes = [P(Params), C.c_void_p, C.c_void_p]
        L.ora_conv_closed_curve.restype = None
        L.ora_conv_closed_curve.argtypes = [C.c_int64, C.c_double, C.c_double, C.c_double,
                                            C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_params(shape, E, lam, model=PC, ps_radius=0, eps=1.0 / 24.0, max_labels=2,
                threads=1, noise=GAUSS, topo=TOPO_OFF, psf_sigma=0.0) -> Params:
    if len(shape) == 2:
        ndim, nz, ny, nx = 2, 1, shape[0], shape[1]
    else:
        ndim, (nz, ny, nx) = 3, shape
    return Params(ndim, nx, ny, nz, model, ps_radius, float(E), float(eps), float(lam),
                  max_labels, threads, noise, topo, float(psf_sigma))


def params_of(w, threads=1) -> Params:
    """Parameters of a workloads.Workload."""
    return make_params(w.image.shape, w.E, w.lam, w.model, w.ps_radius, w.eps,
                       w.max_labels, threads, getattr(w, "noise", GAUSS),
                       getattr(w, "topo", TOPO_OFF), getattr(w, "psf_sigma", 0.0))


def _img(I):
    return np.ascontiguousarray(I, dtype=np.float64)


def _lab(L):
    return np.ascontiguousarray(L, dtype=np.int32)


def kernel(r, E, eps=1.0 / 24.0) -> float:
    return lib().ora_kernel(float(r), float(E), float(eps))


def particles(P: Params, L):
    L = _lab(L)
    n = lib().ora_particles(C.byref(P), _ptr(L), 0, None, None, None)
    lin = np.zeros(n, np.int64)
    a = np.zeros(n, np.int32)
    b = np.zeros(n, np.int32)
    lib().ora_particles(C.byref(P), _ptr(L), n, _ptr(lin), _ptr(a), _ptr(b))
    return lin, a, b


def region_stats(P: Params, I, L):
    M = P.max_labels
    n = np.zeros(M, np.int64)
    s1 = np.zeros(M)
    s2 = np.zeros(M)
    I, L = _img(I), _lab(L)
    lib().ora_region_stats(C.byref(P), _ptr(I), _ptr(L), _ptr(n), _ptr(s1), _ptr(s2))
    return n, s1, s2


def l2diff(P: Params, I, L, lin, a, b):
    I, L = _img(I), _lab(L)
    lin = np.ascontiguousarray(lin, np.int64)
    a = np.ascontiguousarray(a, np.int32)
    b = np.ascontiguousarray(b, np.int32)
    out = np.zeros(len(lin))
    lib().ora_l2diff(C.byref(P), _ptr(I), _ptr(L), len(lin), _ptr(lin), _ptr(a), _ptr(b), _ptr(out))
    return out


def sobolev(P: Params, lin, a, b, dE, neigh=NEIGH_CELLS, sel=None):
    lin = np.ascontiguousarray(lin, np.int64)
    a = np.ascontiguousarray(a, np.int32)
    b = np.ascontiguousarray(b, np.int32)
    dE = np.ascontiguousarray(dE, np.float64)
    if sel is not None:
        sel = np.ascontiguousarray(sel, np.int64)
        out = np.zeros(len(sel))
        lib().ora_sobolev(C.byref(P), len(lin), _ptr(lin), _ptr(a), _ptr(b), _ptr(dE),
                          _ptr(out), neigh, len(sel), _ptr(sel))
    else:
        out = np.zeros(len(lin))
        lib().ora_sobolev(C.byref(P), len(lin), _ptr(lin), _ptr(a), _ptr(b), _ptr(dE),
                          _ptr(out), neigh, 0, None)
    return out


def step(P: Params, I, L, mode=MODE_SOBOLEV, want_arrays=True):
    """One iteration.  Returns (L_next, dict) with the particle list and both
    gradients of the state the step started from."""
    I = _img(I)
    L = _lab(L).copy()
    nf = C.c_int64(0)
    if not want_arrays:
        n = lib().ora_step(C.byref(P), _ptr(I), _ptr(L), mode, 0, None, None, None, None, None,
                           C.byref(nf))
        return L, {"n": n, "flips": nf.value}
    n = lib().ora_particles(C.byref(P), _ptr(L), 0, None, None, None)
    lin = np.zeros(n, np.int64)
    a = np.zeros(n, np.int32)
    b = np.zeros(n, np.int32)
    g2 = np.zeros(n)
    g1 = np.zeros(n)
    r = lib().ora_step(C.byref(P), _ptr(I), _ptr(L), mode, n, _ptr(lin), _ptr(a), _ptr(b),
                       _ptr(g2), _ptr(g1), C.byref(nf))
    assert r == n
    return L, {"n": n, "flips": nf.value, "lin": lin, "a": a, "b": b, "dE_l2": g2, "dE_h1": g1}


def run_ex(P: Params, I, L, mode=MODE_SOBOLEV, max_iters=100, tol=0.0):
    """ora_run with all telemetry: final labels, iterations done, per-iteration
    N_t, flips and reversals, and the first L2 iteration of AUTO mode (-1)."""
    I = _img(I)
    L = _lab(L).copy()
    hn = np.zeros(max_iters, np.int64)
    hf = np.zeros(max_iters, np.int64)
    hb = np.zeros(max_iters, np.int64)
    sw = C.c_int32(-1)
    t = lib().ora_run(C.byref(P), _ptr(I), _ptr(L), mode, max_iters, float(tol), _ptr(hn), _ptr(hf),
                      _ptr(hb), C.byref(sw))
    return {"L": L, "t": t, "n": hn[:t], "flips": hf[:t], "reversals": hb[:t], "switch": sw.value}


def run(P: Params, I, L, mode=MODE_SOBOLEV, max_iters=100, tol=0.0):
    r = run_ex(P, I, L, mode, max_iters, tol)
    return r["L"], r["t"], r["n"], r["flips"]


def simple(P: Params, L, i, label) -> bool:
    """Is pixel i (linear index) a simple point of {L == label}?"""
    L = _lab(L)
    return bool(lib().ora_simple(C.byref(P), _ptr(L), int(i), int(label)))


def accept_ranked(P: Params, L, lin, a, b, g, topo=TOPO_SIMPLE):
    """Ranked acceptance on a copy of L.  Returns (L_next, executed mask, moves)."""
    L = _lab(L).copy()
    lin = np.ascontiguousarray(lin, np.int64)
    a = np.ascontiguousarray(a, np.int32)
    b = np.ascontiguousarray(b, np.int32)
    g = np.ascontiguousarray(g, np.float64)
    done = np.zeros(len(lin), np.uint8)
    m = lib().ora_accept_ranked(C.byref(P), _ptr(L), len(lin), _ptr(lin), _ptr(a), _ptr(b),
                                _ptr(g), int(topo), _ptr(done))
    return L, done.astype(bool), m


def psf_taps(sigma):
    r = lib().ora_psf_radius(float(sigma))
    k = np.zeros(2 * r + 1)
    lib().ora_psf_taps(float(sigma), _ptr(k))
    return k


def deconv_theta(P: Params, I, L):
    th = np.zeros(P.max_labels)
    lib().ora_deconv_theta(C.byref(P), _ptr(_img(I)), _ptr(_lab(L)), _ptr(th))
    return th


def deconv_model(P: Params, L, theta):
    L = _lab(L)
    J = np.zeros(L.shape)
    lib().ora_deconv_model(C.byref(P), _ptr(L), _ptr(np.ascontiguousarray(theta, np.float64)), _ptr(J))
    return J


def reversals(L_prev, L_next, stamp, t):
    """ora_reversals on flat int32 label arrays; stamp (uint32) is updated in place."""
    Lp, Ln = _lab(L_prev), _lab(L_next)
    assert stamp.dtype == np.uint32 and stamp.flags.c_contiguous and stamp.size == Lp.size
    return lib().ora_reversals(Lp.size, _ptr(Lp), _ptr(Ln), _ptr(stamp), int(t))


class AutoRule:
    """ora_auto_init / ora_auto_update: the gradient-mode switch and the stop
    of a run, fed one iteration's (N_t, flips, reversals) at a time."""

    def __init__(self, mode=MODE_AUTO, tol=0.0):
        self.mode, self.tol = int(mode), float(tol)
        self.s = Auto()
        lib().ora_auto_init(C.byref(self.s), self.mode)

    def update(self, n, flips, reversals) -> bool:
        """Iteration t = self.t done; True if the run stops after it."""
        return bool(lib().ora_auto_update(C.byref(self.s), self.mode, self.tol, int(n), int(flips),
                                          int(reversals)))

    @property
    def t(self):
        return self.s.t

    @property
    def grad(self):
        """Gradient mode of the next iteration (MODE_SOBOLEV or MODE_L2)."""
        return self.s.grad

    @property
    def switch_iter(self):
        return self.s.switch_iter


def energy_pc(P: Params, I, L) -> float:
    I, L = _img(I), _lab(L)
    return lib().ora_energy_pc(C.byref(P), _ptr(I), _ptr(L))


def conv_closed_curve(g, Lc, E, eps=1.0 / 24.0):
    g = np.ascontiguousarray(g, np.float64)
    out = np.zeros_like(g)
    lib().ora_conv_closed_curve(len(g), float(Lc), float(E), float(eps), _ptr(g), _ptr(out))
    return out
