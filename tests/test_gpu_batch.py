"""Batched launches (many contexts, one set of launches per iteration) against
stand-alone runs of the same contexts, and against the oracle.

A slot's results must be bit-identical to its stand-alone run: label field,
particle set in context order, region statistics and per-iteration telemetry.
Slots are also checked at every batched iteration against the oracle
stepping from the slot's own labels (particle sets exact, gradients within
1e-5, labels outside the decision margin).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1403_0240_amd import sobrc as S  # noqa: E402
from paper_1403_0240_amd import workloads as W  # noqa: E402
from shadow import Shadow  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.lib()


def small_2d():
    return [W.blobs2d(200 + k, side_lo=40, side_hi=150) for k in range(5)] + [W.disk2d()]


def small_3d():
    return [W.random_multilabel(2, (13, 17, 19), 3, E=6.0, lam=0.5),
            W.random_multilabel(4, (12, 20, 9), 3, dtype=np.uint16, E=6.0, lam=30.0),
            W.half_plane((20, 21, 22), 9, axis=1, E=6.0),
            W.random_multilabel(3, (9, 11, 10), 3, blobs=False, E=6.0, lam=0.2)]


def make_ctx(w):
    cap = max(4096, 2 * w.labels.size)
    ctx, img, lab = S.from_workload(w, max_particles=cap)
    S.init_labels(ctx, img, lab)
    return ctx, img, lab


def snapshot(ctx):
    lin, a, b = (t.cpu().numpy() for t in S.get_particles(ctx))
    n, f, r = S.get_history(ctx, reversals=True)
    cnt, sm = S.get_region_stats(ctx)
    return {"labels": S.get_labels(ctx).cpu().numpy(), "lin": lin, "a": a, "b": b,
            "hist": (n, f, r), "count": cnt, "sum": sm}


def assert_same(x, y, what):
    for k in ("labels", "lin", "a", "b", "count", "sum"):
        assert np.array_equal(x[k], y[k]), f"{what}: {k} differs"
    for u, v in zip(x["hist"], y["hist"]):
        assert np.array_equal(u, v), f"{what}: history differs"


@pytest.mark.parametrize("dims", ["2d", "3d"])
@pytest.mark.parametrize("mode", [S.MODE_SOBOLEV, S.MODE_L2])
def test_batch_equals_standalone(dims, mode):
    ws = small_2d() if dims == "2d" else small_3d()
    print(f"[batch {dims} mode={mode} n={len(ws)}]", flush=True)
    iters = 9  # odd: exercises the graph pairs and one direct step
    solo = []
    for w in ws:
        ctx, _, _ = make_ctx(w)
        assert S.run(ctx, iters, 0.0, mode) == iters
        solo.append(snapshot(ctx))
    B = S.Batch(len(ws) + 1)  # one slot stays empty
    ctxs = [make_ctx(w)[0] for w in ws]
    for k, c in enumerate(ctxs):
        B.set(k + 1 if k >= 2 else k, c)
    done = B.run(iters, 0.0, mode)
    assert done[2] == 0 and all(done[np.arange(len(done)) != 2] == iters)
    for k, c in enumerate(ctxs):
        assert_same(snapshot(c), solo[k], f"slot of image {k}")
    # asynchronous batched steps continue exactly like stand-alone steps
    for _ in range(3):
        B.step(mode)
    for w, c in zip(ws[:2], ctxs[:2]):
        ref, _, _ = make_ctx(w)
        S.run(ref, iters + 3, 0.0, mode)
        assert_same(snapshot(c), snapshot(ref), "after batched steps")
    B.close()


def batch_shadow_steps(ora, B, ctxs, ws, shadowed, iters, mode):
    """iters batched steps; the slots in `shadowed` are checked against the
    oracle at every one."""
    shadows = [Shadow(ora, ws[k], ctxs[k], mode) for k in shadowed]
    for _ in range(iters):
        states = [sh.pre() for sh in shadows]
        B.step(mode)
        for sh, st in zip(shadows, states):
            sh.post(st)
    for k, sh in zip(shadowed, shadows):
        sh.report(f"slot {k}")
        assert sh.checked == iters
    return shadows


@pytest.mark.parametrize("dims", ["2d", "3d"])
@pytest.mark.parametrize("mode", [S.MODE_SOBOLEV, S.MODE_L2])
def test_batch_slots_match_oracle(ora, dims, mode):
    """Three slots of a batch (of different sizes and, in 3D, image types)
    checked against the oracle at each of nine batched iterations."""
    ws = small_2d() if dims == "2d" else small_3d()
    print(f"[batch oracle {dims} mode={mode} n={len(ws)}]", flush=True)
    B = S.Batch(len(ws))
    ctxs = [make_ctx(w)[0] for w in ws]
    for k, c in enumerate(ctxs):
        B.set(k, c)
    batch_shadow_steps(ora, B, ctxs, ws, (0, 1, len(ws) - 1), 9, mode)
    B.close()


@pytest.mark.parametrize("tile", [S.TILE_DEFAULT, S.TILE_WIDE])
def test_batch2d_64_slots_match_oracle(ora, tile):
    """The batched benchmark workload (64 images of 128..1024 pixels a side),
    on the default cells and on the 16x32 cells its benchmark's autotuner
    keeps: the smallest, a middle and the largest image checked against the
    oracle at every one of six batched iterations, with all 64 slots live."""
    ws = W.batch2d()
    ctxs = []
    for w in ws:
        c, img, lab = S.from_workload(w, tile=tile)
        S.init_labels(c, img, lab)
        ctxs.append(c)
    sizes = [w.labels.size for w in ws]
    order = np.argsort(sizes)
    shadowed = (int(order[0]), int(order[len(order) // 2]), int(order[-1]))
    print(f"[batch2d_64 oracle: tile {tile} slots {shadowed}]", flush=True)
    B = S.Batch(len(ws))
    for k, c in enumerate(ctxs):
        B.set(k, c)
    batch_shadow_steps(ora, B, ctxs, ws, shadowed, 6, S.MODE_SOBOLEV)
    B.close()


def test_batch_auto_mode_and_tolerance():
    """Each slot stops on its own tolerance and switches to L2 gradients on its
    own oscillation, as in a stand-alone AUTO run."""
    ws = small_2d()
    print("[batch auto]", flush=True)
    solo, sw = [], []
    for w in ws:
        ctx, _, _ = make_ctx(w)
        t = S.run(ctx, 150, 1e-3, S.MODE_AUTO)
        solo.append((t, snapshot(ctx)))
        sw.append(S.gradient_switch(ctx))
    B = S.Batch(len(ws))
    ctxs = [make_ctx(w)[0] for w in ws]
    for k, c in enumerate(ctxs):
        B.set(k, c)
    done = B.run(150, 1e-3, S.MODE_AUTO)
    for k, c in enumerate(ctxs):
        assert done[k] == solo[k][0]
        assert S.gradient_switch(c) == sw[k]
        assert_same(snapshot(c), solo[k][1], f"auto slot {k}")
    assert len(set(done.tolist())) > 1  # slots really stopped at different iterations
    B.close()


def test_batch_slot_replacement():
    """A slot emptied and refilled mid-run (the serving pattern): the other
    slots are unaffected and the newcomer evolves from its own start."""
    ws = small_2d()
    print("[batch replace]", flush=True)
    B = S.Batch(3)
    a, b, c = (make_ctx(w)[0] for w in ws[:3])
    B.set(0, a)
    B.set(1, b)
    B.run(4, 0.0, S.MODE_SOBOLEV)
    B.set(1, None)
    B.set(2, c)
    B.run(5, 0.0, S.MODE_SOBOLEV)
    for w, ctx, it in ((ws[0], a, 9), (ws[1], b, 4), (ws[2], c, 5)):
        ref, _, _ = make_ctx(w)
        S.run(ref, it, 0.0, S.MODE_SOBOLEV)
        assert_same(snapshot(ctx), snapshot(ref), f"slot context after {it} iterations")
    # b left the batch: it steps on its own again
    assert S.run(b, 2, 0.0, S.MODE_SOBOLEV) == 2
    B.close()


def test_batch_errors():
    ws = small_2d()
    B = S.Batch(2)
    a, _, _ = make_ctx(ws[0])
    B.set(0, a)
    with pytest.raises(S.SobrcError) as e:
        S.step(a)
    assert e.value.code == S.ESTATE
    with pytest.raises(S.SobrcError) as e:
        S.run(a, 1)
    assert e.value.code == S.ESTATE
    w3 = small_3d()[0]
    c3, _, _ = make_ctx(w3)
    with pytest.raises(S.SobrcError) as e:
        B.set(1, c3)  # other ndim / E
    assert e.value.code == S.EINVAL
    wE = W.blobs2d(300, side_lo=40, side_hi=80, E=12.0)
    cE, _, _ = make_ctx(wE)
    with pytest.raises(S.SobrcError) as e:
        B.set(1, cE)
    assert e.value.code == S.EINVAL
    with pytest.raises(S.SobrcError) as e:
        B.set(1, a)  # already in slot 0
    assert e.value.code == S.ESTATE
    B.close()
    assert S.run(a, 1) == 1  # released by close


@pytest.mark.parametrize("dims", ["2d", "3d"])
def test_launch_shapes_do_not_change_results(dims):
    """Launch shapes regroup work only: the autotuner's trial iterations and
    extreme shapes leave every slot on its stand-alone trajectory."""
    ws = small_2d() if dims == "2d" else small_3d()
    print(f"[batch shapes {dims}]", flush=True)
    B = S.Batch(len(ws))
    ctxs = [make_ctx(w)[0] for w in ws]
    for k, c in enumerate(ctxs):
        B.set(k, c)
    shape, tuned = B.autotune(S.MODE_SOBOLEV, iters_per_trial=1)
    assert tuned >= 2
    total = tuned
    for sh in [(64, 8, 1), (1 << 20, 8, 1 << 20), (0, 0, 0), shape]:
        B.set_shape(*sh)
        done = B.run(3, 0.0, S.MODE_SOBOLEV)
        assert (done == 3).all()
        total += 3
    for w, c in zip(ws, ctxs):
        ref, _, _ = make_ctx(w)
        assert S.run(ref, total, 0.0, S.MODE_SOBOLEV) == total
        assert_same(snapshot(c), snapshot(ref), f"after {total} iterations over several shapes")
    B.close()


@pytest.mark.parametrize("dims", ["2d", "3d"])
def test_wide_tiles_batch_equals_standalone(dims):
    """Contexts with wide cells batch like any others (each slot on its
    stand-alone trajectory), and a batch refuses a context of the other cell
    shape."""
    ws = small_2d() if dims == "2d" else small_3d()
    for w in ws:
        w.tile = S.TILE_WIDE
    print(f"[batch wide tiles {dims}]", flush=True)
    B = S.Batch(len(ws) + 1)
    ctxs = [make_ctx(w)[0] for w in ws]
    for k, c in enumerate(ctxs):
        B.set(k, c)
    done = B.run(6, 0.0, S.MODE_SOBOLEV)
    assert (done[: len(ws)] == 6).all()
    for w, c in zip(ws, ctxs):
        ref, _, _ = make_ctx(w)
        assert S.run(ref, 6, 0.0, S.MODE_SOBOLEV) == 6
        assert_same(snapshot(c), snapshot(ref), "wide cells, batch against stand-alone")
    w0 = ws[0]
    w0.tile = S.TILE_DEFAULT
    other, _, _ = make_ctx(w0)
    with pytest.raises(S.SobrcError) as e:
        B.set(len(ws), other)
    assert e.value.code == S.EINVAL
    B.close()


def test_batch_mixes_likelihoods():
    """Slots with Poisson noise, the piecewise-smooth model or more than 16
    labels (region sums by atomics) run in the same batch as Gaussian
    piecewise-constant slots, each equal to its own run."""
    ws = [W.random_multilabel(22, (30, 34), 3, E=6.0, lam=0.5, model=W.PS, ps_radius=3, noise=W.POISSON),
          W.random_multilabel(23, (27, 41), 3, E=6.0, lam=0.7, noise=W.POISSON),
          W.blobs2d(210, side_lo=40, side_hi=120, E=6.0),
          W.random_multilabel(43, (44, 50), 24, E=6.0, lam=0.3)]
    print(f"[batch likelihood mix n={len(ws)}]", flush=True)
    iters = 7
    solo = []
    for w in ws:
        ctx, _, _ = make_ctx(w)
        assert S.run(ctx, iters, 0.0, S.MODE_SOBOLEV) == iters
        solo.append(snapshot(ctx))
    B = S.Batch(len(ws))
    ctxs = [make_ctx(w)[0] for w in ws]
    for k, c in enumerate(ctxs):
        B.set(k, c)
    done = B.run(iters, 0.0, S.MODE_SOBOLEV)
    assert all(done == iters)
    for k, c in enumerate(ctxs):
        assert_same(snapshot(c), solo[k], f"slot of image {k}")
    B.close()
