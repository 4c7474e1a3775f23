"""Python binding of libsobrc.so (C ABI in include/sobrc.h).

Argument marshalling only: torch tensors provide device memory, torch's current
HIP stream is passed through; every step of the computation runs in the HIP
kernels of the library.  Importing works without a GPU; any call that reaches
the device needs the built library and a GPU, and fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsobrc.so")

OK, EINVAL, ECAPACITY, EDEVICE, ESTATE = 0, -1, -2, -3, -4
F32, U16 = 0, 1
PC, PS = 0, 1
NOISE_GAUSS, NOISE_POISSON = 0, 1
MODE_SOBOLEV, MODE_L2, MODE_AUTO = 0, 1, 2
TOPO_OFF, TOPO_SIMPLE = 0, 1
TILE_DEFAULT, TILE_WIDE, TILE_TALL = 0, 1, 2
K_L2DIFF, K_SOBOLEV, K_FLIP, K_COUNT, K_SCAN, K_WRITE, K_TOPO, K_DECONV = range(8)
KERNEL_NAMES = ("k_l2diff", "k_sobolev", "k_flip", "k_count", "k_scan", "k_write", "k_topo",
                "k_deconv")

EXPORTS = ("workspace_size", "ctx_create", "ctx_destroy", "init_labels", "compute_l2_diff",
           "sobolev_smooth", "step", "step_with_gradient", "run", "ctx_sync", "get_particles", "get_labels",
           "get_labels_u16", "tile_autotune_workspace_size", "tile_autotune",
           "get_region_stats", "get_history", "get_gradient_mode", "sobolev_particles_workspace_size",
           "sobolev_smooth_particles", "sobolev_smooth_particles_static", "profile_enable", "profile_read", "batch_workspace_size",
           "batch_create", "batch_destroy", "batch_set", "batch_step", "batch_run",
           "batch_launch_iters", "batch_collect", "batch_set_shape", "batch_autotune", "last_error")


class SobrcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sobrc error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("image_dtype", C.c_int32), ("model", C.c_int32), ("ps_radius", C.c_int32),
        ("E", C.c_double), ("eps", C.c_double), ("lam", C.c_double),
        ("max_labels", C.c_int32), ("max_particles", C.c_int64), ("noise", C.c_int32),
        ("topo", C.c_int32), ("psf_sigma", C.c_double), ("tile", C.c_int32),
    ]


_lib = None


def lib():
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    P, V, I32, I64 = C.POINTER, C.c_void_p, C.c_int32, C.c_int64
    sig = {
        "workspace_size": [P(Params), P(C.c_size_t)],
        "ctx_create": [P(Params), V, C.c_size_t, P(V)],
        "ctx_destroy": [V],
        "init_labels": [V, V, V, V],
        "compute_l2_diff": [V, V, V],
        "sobolev_smooth": [V, V, V, V],
        "step": [V, I32, V, V],
        "step_with_gradient": [V, V, V, V],
        "run": [V, I32, C.c_double, I32, P(I32), V],
        "ctx_sync": [V, V],
        "get_particles": [V, P(I64), V, V, V, V],
        "get_labels": [V, V, V],
        "get_labels_u16": [V, V, V],
        "tile_autotune_workspace_size": [P(Params), P(C.c_size_t)],
        "tile_autotune": [P(Params), V, V, I32, I32, V, C.c_size_t, P(I32), V, V],
        "get_region_stats": [V, V, V, V],
        "get_history": [V, I32, V, V, V, P(I32), V],
        "get_gradient_mode": [V, P(I32), V],
        "sobolev_particles_workspace_size": [P(Params), I64, P(C.c_size_t)],
        "sobolev_smooth_particles": [P(Params), I64, V, V, V, V, V, V, C.c_size_t, V],
        "sobolev_smooth_particles_static": [P(Params), I64, V, V, V, V, V, V],
        "profile_enable": [V, I32],
        "profile_read": [V, V, V, I32],
        "batch_workspace_size": [I32, P(C.c_size_t)],
        "batch_create": [I32, V, C.c_size_t, P(V)],
        "batch_destroy": [V],
        "batch_set": [V, I32, V, V],
        "batch_step": [V, I32, V],
        "batch_run": [V, I32, C.c_double, I32, V, V],
        "batch_launch_iters": [V, I32, C.c_double, I32, V],
        "batch_collect": [V, V, V, V],
        "batch_set_shape": [V, I32, I32, I32, V],
        "batch_autotune": [V, I32, I32, V, V, V],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = I32
    L.last_error.argtypes = []
    L.last_error.restype = C.c_char_p
    _lib = L
    return L


def _check(code: int):
    if code != OK:
        raise SobrcError(code, lib().last_error().decode(errors="replace"))


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def make_params(shape, image_dtype, E, lam, model=PC, ps_radius=0, eps=1.0 / 24.0,
                max_labels=2, max_particles=1 << 20, noise=0, topo=TOPO_OFF, psf_sigma=0.0,
                tile=0) -> Params:
    """Parameters for an image of numpy-style shape (ny, nx) or (nz, ny, nx)."""
    if len(shape) == 2:
        ndim, nz, ny, nx = 2, 1, shape[0], shape[1]
    else:
        ndim, (nz, ny, nx) = 3, shape
    dt = U16 if image_dtype in (torch.uint16, "uint16", U16) else F32
    return Params(ndim, nx, ny, nz, dt, model, ps_radius, float(E), float(eps), float(lam),
                  max_labels, int(max_particles), int(noise), int(topo), float(psf_sigma), int(tile))


def workspace_size(params: Params) -> int:
    n = C.c_size_t(0)
    _check(lib().workspace_size(C.byref(params), C.byref(n)))
    return n.value


class Context:
    """A segmentation job: device workspace + library context.

    ``image`` must be a contiguous CUDA (HIP) tensor of float32 or uint16 with
    the shape given in ``params``; the context keeps a reference to it."""

    def __init__(self, params: Params, device="cuda"):
        self.params = params
        self.nbytes = workspace_size(params)
        self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        h = C.c_void_p(0)
        _check(lib().ctx_create(C.byref(params), _ptr(self.workspace), self.nbytes, C.byref(h)))
        self.handle = h
        self.image = None
        self.shape = ((params.ny, params.nx) if params.ndim == 2
                      else (params.nz, params.ny, params.nx))

    def close(self):
        if self.handle:
            lib().ctx_destroy(self.handle)
            self.handle = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def device(self):
        return self.workspace.device


def ctx_create(params: Params, device="cuda") -> Context:
    return Context(params, device)


def ctx_destroy(ctx: Context):
    ctx.close()


def _dev_tensor(t, dtype, shape, what):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{what} must be a contiguous {dtype} tensor on the GPU")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def init_labels(ctx: Context, image: torch.Tensor, labels: torch.Tensor, stream=None):
    dt = torch.uint16 if ctx.params.image_dtype == U16 else torch.float32
    _dev_tensor(image, dt, ctx.shape, "image")
    _dev_tensor(labels, torch.int32, ctx.shape, "labels")
    ctx.image = image
    _check(lib().init_labels(ctx.handle, _ptr(image), _ptr(labels), _stream(stream)))


def _cap_tensor(ctx, out):
    if out is None:
        out = torch.empty(ctx.params.max_particles, dtype=torch.float32, device=ctx.device)
    elif not (out.is_cuda and out.dtype == torch.float32 and out.numel() >= ctx.params.max_particles):
        raise ValueError("output must be a float32 GPU tensor with max_particles entries")
    return out


def compute_l2_diff(ctx: Context, out=None, stream=None) -> torch.Tensor:
    """L2 gradient of the current particles (first n entries valid)."""
    out = _cap_tensor(ctx, out)
    _check(lib().compute_l2_diff(ctx.handle, _ptr(out), _stream(stream)))
    return out


def sobolev_smooth(ctx: Context, inp: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    out = _cap_tensor(ctx, out)
    if not (inp.is_cuda and inp.dtype == torch.float32):
        raise ValueError("input must be a float32 GPU tensor")
    _check(lib().sobolev_smooth(ctx.handle, _ptr(inp), _ptr(out), _stream(stream)))
    return out


def step(ctx: Context, mode=MODE_SOBOLEV, nflips: torch.Tensor | None = None, stream=None):
    _check(lib().step(ctx.handle, mode, _ptr(nflips), _stream(stream)))


def step_with_gradient(ctx: Context, grad: torch.Tensor, nflips: torch.Tensor | None = None, stream=None):
    """One iteration driven by a caller-supplied fp32 gradient (device tensor,
    one value per current particle in context order)."""
    if grad.dtype != torch.float32 or not grad.is_cuda or not grad.is_contiguous():
        raise ValueError("grad must be a contiguous float32 device tensor")
    if grad.numel() < particle_count(ctx, stream):
        raise ValueError("grad needs one value per current particle")
    _check(lib().step_with_gradient(ctx.handle, _ptr(grad), _ptr(nflips), _stream(stream)))


def run(ctx: Context, max_iters: int, flip_tol: float = 0.0, mode=MODE_SOBOLEV, stream=None) -> int:
    done = C.c_int32(0)
    _check(lib().run(ctx.handle, max_iters, float(flip_tol), mode, C.byref(done), _stream(stream)))
    return done.value


def ctx_sync(ctx: Context, stream=None):
    _check(lib().ctx_sync(ctx.handle, _stream(stream)))


def particle_count(ctx: Context, stream=None) -> int:
    n = C.c_int64(0)
    _check(lib().get_particles(ctx.handle, C.byref(n), None, None, None, _stream(stream)))
    return n.value


def get_particles(ctx: Context, stream=None):
    """(lin, a, b) int32 tensors of the current particles in context order."""
    n = particle_count(ctx, stream)
    lin = torch.empty(max(n, 1), dtype=torch.int32, device=ctx.device)
    a = torch.empty_like(lin)
    b = torch.empty_like(lin)
    m = C.c_int64(0)
    _check(lib().get_particles(ctx.handle, C.byref(m), _ptr(lin), _ptr(a), _ptr(b), _stream(stream)))
    return lin[:n], a[:n], b[:n]


def get_labels(ctx: Context, out=None, stream=None) -> torch.Tensor:
    if out is None:
        out = torch.empty(ctx.shape, dtype=torch.int32, device=ctx.device)
    _dev_tensor(out, torch.int32, ctx.shape, "labels")
    _check(lib().get_labels(ctx.handle, _ptr(out), _stream(stream)))
    return out


def get_labels_u16(ctx: Context, out=None, stream=None) -> torch.Tensor:
    """The label field as the context holds it (uint16) in `out`: a device tensor or a
    page-locked host tensor (one asynchronous copy on `stream`; synchronise before reading
    a host tensor).  Default: a new device tensor."""
    if out is None:
        out = torch.empty(ctx.shape, dtype=torch.uint16, device=ctx.device)
    ok = (isinstance(out, torch.Tensor) and out.dtype == torch.uint16 and out.is_contiguous()
          and (out.is_cuda or out.is_pinned()))
    if not ok:
        raise ValueError("labels must be a contiguous uint16 tensor on the GPU or in page-locked host memory")
    if tuple(out.shape) != tuple(ctx.shape):
        raise ValueError(f"labels has shape {tuple(out.shape)}, expected {tuple(ctx.shape)}")
    _check(lib().get_labels_u16(ctx.handle, _ptr(out), _stream(stream)))
    return out


def tile_autotune(params: Params, image, labels, iters: int = 4, mode=MODE_SOBOLEV, stream=None):
    """Time `iters` iterations with each cell shape on this image (device
    tensors as for init_labels); returns (chosen TILE_*, [ms per iteration of
    TILE_DEFAULT, TILE_WIDE, TILE_TALL]) (-1 for a shape the parameters do not
    admit)."""
    nb = C.c_size_t(0)
    _check(lib().tile_autotune_workspace_size(C.byref(params), C.byref(nb)))
    ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=image.device)
    tile = C.c_int32(0)
    ms = (C.c_double * 3)()
    _check(lib().tile_autotune(C.byref(params), _ptr(image), _ptr(labels), int(iters), mode, _ptr(ws),
                               nb.value, C.byref(tile), ms, _stream(stream)))
    return tile.value, [ms[0], ms[1], ms[2]]


def get_region_stats(ctx: Context, stream=None):
    import numpy as np
    M = ctx.params.max_labels
    n = np.zeros(M, np.int64)
    s = np.zeros(M, np.float64)
    _check(lib().get_region_stats(ctx.handle, n.ctypes.data_as(C.c_void_p),
                                  s.ctypes.data_as(C.c_void_p), _stream(stream)))
    return n, s


def get_history(ctx: Context, cap: int = 4096, stream=None, reversals=False):
    """(N_t, flips_t) of the most recent iterations, oldest first; with
    reversals=True also reversals_t."""
    import numpy as np
    hn = np.zeros(cap, np.int32)
    hf = np.zeros(cap, np.int32)
    hb = np.zeros(cap, np.int32)
    ln = C.c_int32(0)
    _check(lib().get_history(ctx.handle, cap, hn.ctypes.data_as(C.c_void_p),
                             hf.ctypes.data_as(C.c_void_p), hb.ctypes.data_as(C.c_void_p),
                             C.byref(ln), _stream(stream)))
    k = ln.value
    return (hn[:k], hf[:k], hb[:k]) if reversals else (hn[:k], hf[:k])


def gradient_switch(ctx: Context, stream=None) -> int:
    """First iteration (since init_labels) run with L2 gradients in AUTO mode, or -1."""
    it = C.c_int32(0)
    _check(lib().get_gradient_mode(ctx.handle, C.byref(it), _stream(stream)))
    return it.value


def sobolev_smooth_particles(params: Params, lin, a, b, inp, out=None, stream=None):
    """Stateless Eq. (6) on caller-given particles (int32 lin/a/b, float32 values)."""
    n = int(lin.numel())
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=lin.device)
    nb = C.c_size_t(0)
    _check(lib().sobolev_particles_workspace_size(C.byref(params), n, C.byref(nb)))
    ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=lin.device)
    _check(lib().sobolev_smooth_particles(C.byref(params), n, _ptr(lin), _ptr(a), _ptr(b),
                                          _ptr(inp), _ptr(out), _ptr(ws), nb.value, _stream(stream)))
    return out


def sobolev_smooth_particles_static(params: Params, lin, a, b, inp, out, stream=None):
    """sobolev_smooth_particles with the library's static scratch memory:
    allocates nothing (the caller provides the output)."""
    n = int(lin.numel())
    _check(lib().sobolev_smooth_particles_static(C.byref(params), n, _ptr(lin), _ptr(a), _ptr(b),
                                                 _ptr(inp), _ptr(out), _stream(stream)))
    return out


def profile_enable(ctx: Context, on: bool = True):
    _check(lib().profile_enable(ctx.handle, 1 if on else 0))


def profile_read(ctx: Context, reset: bool = True):
    """{kernel name: (total ms, launches)} since the last reset."""
    import numpy as np
    nk = len(KERNEL_NAMES)  # SOBRC_K_NKINDS
    ms = np.zeros(nk, np.float64)
    n = np.zeros(nk, np.int64)
    _check(lib().profile_read(ctx.handle, ms.ctypes.data_as(C.c_void_p),
                              n.ctypes.data_as(C.c_void_p), 1 if reset else 0))
    return {KERNEL_NAMES[k]: (float(ms[k]), int(n[k])) for k in range(nk)}


def workload_params(w, max_particles=None, tile=None) -> Params:
    """Params of a workloads.Workload (tile None: the workload's own)."""
    import numpy as np
    if max_particles is None:
        max_particles = default_capacity(w.image.shape)
    dt = U16 if w.image.dtype == np.uint16 else F32
    return make_params(w.image.shape, dt, w.E, w.lam, w.model, w.ps_radius, w.eps,
                       w.max_labels, max_particles, getattr(w, "noise", 0), getattr(w, "topo", 0),
                       getattr(w, "psf_sigma", 0.0), getattr(w, "tile", 0) if tile is None else tile)


def workload_tensors(w, device="cuda"):
    """The workload's image and initial labels as contiguous device tensors."""
    import numpy as np
    if w.image.dtype == np.uint16:
        img = torch.from_numpy(np.ascontiguousarray(w.image, np.uint16)).to(device)
    else:
        img = torch.from_numpy(np.ascontiguousarray(w.image, np.float32)).to(device)
    lab = torch.from_numpy(np.ascontiguousarray(w.labels, np.int32)).to(device)
    return img.contiguous(), lab.contiguous()


def from_workload(w, max_particles=None, device="cuda", tile=None):
    """Context + device tensors for a workloads.Workload; returns (ctx, image, labels).
    tile: TILE_DEFAULT / TILE_WIDE (None: the workload's own)."""
    ctx = Context(workload_params(w, max_particles, tile), device)
    img, lab = workload_tensors(w, device)
    return ctx, img, lab


def default_capacity(shape) -> int:
    """A particle capacity generous for smooth contours: a quarter of the
    pixels, at least 4096."""
    n = 1
    for s in shape:
        n *= int(s)
    return int(min(max(n // 4, 4096), 0x7fffffff))


class Batch:
    """A table of slots, each empty or holding an initialised Context; all
    live slots advance together, one set of launches per iteration.  Keeps a
    reference to every context in a slot."""

    def __init__(self, n_slots: int, device="cuda"):
        nb = C.c_size_t(0)
        _check(lib().batch_workspace_size(n_slots, C.byref(nb)))
        self.n_slots = n_slots
        self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=device)
        h = C.c_void_p(0)
        _check(lib().batch_create(n_slots, _ptr(self.workspace), nb.value, C.byref(h)))
        self.handle = h
        self.slots = [None] * n_slots

    def set(self, slot: int, ctx: "Context | None", stream=None):
        _check(lib().batch_set(self.handle, slot, ctx.handle if ctx is not None else None,
                               _stream(stream)))
        self.slots[slot] = ctx

    def step(self, mode=MODE_SOBOLEV, stream=None):
        _check(lib().batch_step(self.handle, mode, _stream(stream)))

    def run(self, max_iters: int, flip_tol: float = 0.0, mode=MODE_SOBOLEV, stream=None):
        """Iterations done per slot (numpy int32, 0 for empty slots)."""
        import numpy as np
        done = np.zeros(self.n_slots, np.int32)
        _check(lib().batch_run(self.handle, max_iters, float(flip_tol), mode,
                               done.ctypes.data_as(C.c_void_p), _stream(stream)))
        return done

    def launch(self, iters: int, flip_tol: float = 0.0, mode=MODE_SOBOLEV, stream=None):
        """Enqueue iterations without synchronising (see collect)."""
        _check(lib().batch_launch_iters(self.handle, iters, float(flip_tol), mode, _stream(stream)))

    def collect(self, stream=None, slot_errors=False):
        """Synchronise; per slot: iterations since init_labels and stopped flag
        (tolerance met or an error).  With slot_errors=True a slot's own error
        does not raise: the second array then holds each slot's state code
        (0 running, 1 stopped at its tolerance, a negative error code)."""
        import numpy as np
        it = np.zeros(self.n_slots, np.int32)
        st = np.zeros(self.n_slots, np.int32)
        code = lib().batch_collect(self.handle, it.ctypes.data_as(C.c_void_p),
                                   st.ctypes.data_as(C.c_void_p), _stream(stream))
        if code != OK and not (slot_errors and (st == code).any()):
            _check(code)
        return (it, st) if slot_errors else (it, st != 0)

    def set_shape(self, part_chunk=0, lg_range=0, sob_tiles=0, stream=None):
        _check(lib().batch_set_shape(self.handle, part_chunk, lg_range, sob_tiles, _stream(stream)))

    def autotune(self, mode=MODE_SOBOLEV, iters_per_trial=2, stream=None):
        """Returns (chosen shape, iterations run)."""
        import numpy as np
        shape = np.zeros(3, np.int32)
        done = C.c_int32(0)
        _check(lib().batch_autotune(self.handle, mode, iters_per_trial,
                                    shape.ctypes.data_as(C.c_void_p), C.byref(done), _stream(stream)))
        return tuple(int(v) for v in shape), done.value

    def close(self):
        if self.handle:
            lib().batch_destroy(self.handle)
            self.handle = C.c_void_p(0)
            self.slots = [None] * self.n_slots

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
