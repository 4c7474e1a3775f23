"""C-ABI contract checks that run without a GPU: the library loads, exports
every function include/sobrc.h declares, and rejects bad parameters and call
orders on the host before touching the device."""
import ctypes as C
import os
import re

import pytest

from paper_1403_0240_amd import sobrc as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sobrc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int32_t|const char\*)\s+(\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(S.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return S.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(S.EXPORTS)


def _p(**kw):
    p = S.make_params((64, 48), "float32", 8.0, 0.1, max_particles=1000)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("kw", [dict(ndim=4), dict(nx=0), dict(ny=40000), dict(nz=2),
                                dict(image_dtype=7), dict(model=3), dict(model=S.PS, ps_radius=1),
                                dict(E=0.0), dict(E=65.0), dict(eps=0.0), dict(lam=-1.0),
                                dict(max_labels=1), dict(max_labels=65536), dict(max_particles=0),
                                dict(noise=2), dict(noise=-1), dict(topo=2), dict(topo=-1),
                                dict(psf_sigma=-1.0), dict(psf_sigma=16.5),
                                dict(psf_sigma=2.0, model=S.PS, ps_radius=3),
                                dict(psf_sigma=2.0, noise=S.NOISE_POISSON),
                                dict(psf_sigma=2.0, max_labels=5), dict(tile=3), dict(tile=-1),
                                dict(tile=S.TILE_WIDE, topo=S.TOPO_SIMPLE),
                                dict(tile=S.TILE_TALL, topo=S.TOPO_SIMPLE)])
def test_bad_params(L, kw):
    n = C.c_size_t(0)
    assert L.workspace_size(C.byref(_p(**kw)), C.byref(n)) == S.EINVAL
    assert L.last_error()


def test_tile_shapes(L):
    """Wide cells: the same label field and tile-major copies in fewer, longer
    tiles; the autotuner's scratch covers both shapes, and it validates its
    arguments on the host."""
    for shape in [(64, 48), (9, 40, 33)]:
        d = S.make_params(shape, "float32", 6.0, 0.1, max_particles=1000)
        w = S.make_params(shape, "float32", 6.0, 0.1, max_particles=1000, tile=S.TILE_WIDE)
        nd, nw, na = C.c_size_t(0), C.c_size_t(0), C.c_size_t(0)
        assert L.workspace_size(C.byref(d), C.byref(nd)) == S.OK
        assert L.workspace_size(C.byref(w), C.byref(nw)) == S.OK
        assert L.tile_autotune_workspace_size(C.byref(w), C.byref(na)) == S.OK
        sizes = [nd.value, nw.value]
        if len(shape) == 2:
            t = S.make_params(shape, "float32", 6.0, 0.1, max_particles=1000, tile=S.TILE_TALL)
            nt = C.c_size_t(0)
            assert L.workspace_size(C.byref(t), C.byref(nt)) == S.OK
            sizes.append(nt.value)
        else:
            t = S.make_params(shape, "float32", 6.0, 0.1, max_particles=1000, tile=S.TILE_TALL)
            assert L.workspace_size(C.byref(t), C.byref(C.c_size_t())) == S.EINVAL  # 2D only
        assert na.value == max(sizes)
    t = S.make_params((9, 40, 33), "float32", 6.0, 0.1, max_particles=1000, topo=S.TOPO_SIMPLE)
    nt, na = C.c_size_t(0), C.c_size_t(0)
    assert L.workspace_size(C.byref(t), C.byref(nt)) == S.OK
    assert L.tile_autotune_workspace_size(C.byref(t), C.byref(na)) == S.OK
    assert na.value == nt.value  # the wide shape is not tried with topological control
    fake = C.c_void_p(1 << 20)  # never dereferenced: rejected before any device call
    tile, ms = C.c_int32(0), (C.c_double * 3)()
    ta = L.tile_autotune
    assert ta(None, fake, fake, 4, 0, fake, 1 << 20, C.byref(tile), ms, None) == S.EINVAL
    assert ta(C.byref(w), None, fake, 4, 0, fake, 1 << 20, C.byref(tile), ms, None) == S.EINVAL
    assert ta(C.byref(w), fake, fake, 0, 0, fake, 1 << 20, C.byref(tile), ms, None) == S.EINVAL
    assert ta(C.byref(w), fake, fake, 4, 7, fake, 1 << 20, C.byref(tile), ms, None) == S.EINVAL
    assert ta(C.byref(w), fake, fake, 4, 0, fake, 1 << 20, None, ms, None) == S.EINVAL


def test_3d_limits(L):
    p = S.make_params((8, 2000, 16), "uint16", 6.0, 1.0)
    assert L.workspace_size(C.byref(p), C.byref(C.c_size_t())) == S.EINVAL
    p = S.make_params((1024, 1024, 1024), "uint16", 6.0, 1.0, max_particles=1 << 24)
    n = C.c_size_t(0)
    assert L.workspace_size(C.byref(p), C.byref(n)) == S.OK
    assert n.value > 2 * 1024 ** 3  # u16 label field


def test_workspace_grows_with_capacity(L):
    a, b = C.c_size_t(0), C.c_size_t(0)
    assert L.workspace_size(C.byref(_p(max_particles=1000)), C.byref(a)) == 0
    assert L.workspace_size(C.byref(_p(max_particles=100000)), C.byref(b)) == 0
    assert b.value - a.value >= 99000 * 23  # records x2, gradients x2


def test_topology_workspace(L):
    """Topological control adds an 8-byte word per pixel and a state byte
    per particle (plus per-tile marks)."""
    a, b = C.c_size_t(0), C.c_size_t(0)
    assert L.workspace_size(C.byref(_p()), C.byref(a)) == 0
    assert L.workspace_size(C.byref(_p(topo=S.TOPO_SIMPLE)), C.byref(b)) == 0
    assert b.value - a.value >= 64 * 48 * 8 + 1000


def test_psf_workspace(L):
    """The deconvolving model adds (max_labels + 4) images of fp32."""
    a, b = C.c_size_t(0), C.c_size_t(0)
    assert L.workspace_size(C.byref(_p(max_labels=3)), C.byref(a)) == 0
    assert L.workspace_size(C.byref(_p(max_labels=3, psf_sigma=2.0)), C.byref(b)) == 0
    assert b.value - a.value >= 64 * 48 * 4 * 7


def test_call_order_and_nulls(L):
    p = _p()
    n = C.c_size_t(0)
    assert L.workspace_size(C.byref(p), C.byref(n)) == 0
    h = C.c_void_p(0)
    fake = C.c_void_p(1 << 20)  # never dereferenced: ctx_create makes no device call
    assert L.ctx_create(C.byref(p), None, n.value, C.byref(h)) == S.EINVAL
    assert L.ctx_create(C.byref(p), C.c_void_p((1 << 20) + 4), n.value, C.byref(h)) == S.EINVAL
    assert L.ctx_create(C.byref(p), fake, n.value - 1, C.byref(h)) == S.EINVAL
    assert L.ctx_create(C.byref(p), fake, n.value, C.byref(h)) == S.OK
    try:
        assert L.step(h, S.MODE_SOBOLEV, None, None) == S.ESTATE
        assert L.step_with_gradient(h, fake, None, None) == S.ESTATE
        assert L.step_with_gradient(None, fake, None, None) == S.EINVAL
        assert L.run(h, 3, 0.0, S.MODE_SOBOLEV, None, None) == S.ESTATE
        assert L.compute_l2_diff(h, fake, None) == S.ESTATE
        assert L.sobolev_smooth(h, fake, fake, None) == S.ESTATE
        assert L.get_labels(h, fake, None) == S.ESTATE
        assert L.get_labels_u16(h, fake, None) == S.ESTATE
        assert L.get_labels_u16(h, None, None) == S.EINVAL
        assert L.get_particles(h, C.byref(C.c_int64()), None, None, None, None) == S.ESTATE
        assert L.ctx_sync(h, None) == S.ESTATE
        assert L.init_labels(h, None, fake, None) == S.EINVAL
        assert L.init_labels(None, fake, fake, None) == S.EINVAL
        assert L.last_error()
    finally:
        assert L.ctx_destroy(h) == S.OK
    assert L.ctx_destroy(None) == S.EINVAL


def test_stateless_validation(L):
    p = _p()
    n = C.c_size_t(0)
    assert L.sobolev_particles_workspace_size(C.byref(p), -1, C.byref(n)) == S.EINVAL
    assert L.sobolev_particles_workspace_size(C.byref(p), 10, C.byref(n)) == S.OK
    # zero particles: nothing to do, no device call
    assert L.sobolev_smooth_particles(C.byref(p), 0, None, None, None, None, None, None, 0, None) == S.OK
    fake = C.c_void_p(1 << 20)
    assert L.sobolev_smooth_particles(C.byref(p), 10, fake, fake, fake, fake, fake, fake, 16, None) == S.EINVAL


def test_static_scratch_validation(L):
    """The no-allocation stateless entry point checks its arguments and its
    scratch limit on the host, before any device call."""
    p = _p()
    fake = C.c_void_p(1 << 20)
    sp = L.sobolev_smooth_particles_static
    assert sp(C.byref(p), 0, None, None, None, None, None, None) == S.OK  # nothing to do
    assert sp(None, 10, fake, fake, fake, fake, fake, None) == S.EINVAL
    assert sp(C.byref(p), -1, fake, fake, fake, fake, fake, None) == S.EINVAL
    assert sp(C.byref(p), 10, None, fake, fake, fake, fake, None) == S.EINVAL
    # more particles than the static scratch holds
    n = C.c_size_t(0)
    big = 4 << 20
    assert L.sobolev_particles_workspace_size(C.byref(p), big, C.byref(n)) == S.OK and n.value > 32 << 20
    assert sp(C.byref(p), big, fake, fake, fake, fake, fake, None) == S.EINVAL
    assert b"static" in L.last_error()


def test_batch_validation(L):
    """Batch entry points reject bad arguments on the host."""
    nb = C.c_size_t(0)
    assert L.batch_workspace_size(0, C.byref(nb)) == S.EINVAL
    assert L.batch_workspace_size(4, None) == S.EINVAL
    assert L.batch_workspace_size(4, C.byref(nb)) == S.OK and nb.value >= 4 * 256
    small = C.c_size_t(0)
    L.batch_workspace_size(1, C.byref(small))
    assert 0 < small.value < nb.value
    h = C.c_void_p(0)
    assert L.batch_create(4, None, nb.value, C.byref(h)) == S.EINVAL
    assert L.batch_create(4, C.c_void_p(0x1001), nb.value, C.byref(h)) == S.EINVAL  # misaligned
    assert L.batch_create(4, C.c_void_p(0x10000), 16, C.byref(h)) == S.EINVAL  # too small
    assert L.batch_create(4, C.c_void_p(0x10000), nb.value, None) == S.EINVAL
    assert not h.value
    for rc in (L.batch_destroy(None), L.batch_set(None, 0, None, None), L.batch_step(None, 0, None),
               L.batch_run(None, 1, 0.0, 0, None, None)):
        assert rc == S.EINVAL
    assert b"batch" in L.last_error()
