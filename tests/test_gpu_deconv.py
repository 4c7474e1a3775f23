"""Deconvolving image model on the GPU (params.psf_sigma > 0), through the C
ABI, against the oracle (direct-summation convolutions, FP64).

Bars as in test_gpu_parity: particle sets bit-exact, L2 and Sobolev gradients
within max |gpu - oracle| <= 1e-5 max |oracle|, labels after a step identical
outside the margin.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1403_0240_amd import sobrc as S  # noqa: E402
from paper_1403_0240_amd import workloads as W  # noqa: E402
from shadow import REL_GRAD, Shadow, match_order, rel_err  # noqa: E402


def gpu_state(w, cap=None):
    ctx, img, lab = S.from_workload(w, max_particles=cap)
    S.init_labels(ctx, img, lab)
    return ctx, img, lab


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.lib()


def _case(seed, shape, sigma, n_labels=3, lam=0.3, dtype=np.float32):
    w = W.random_multilabel(seed, shape, n_labels, E=6.0, lam=lam, dtype=dtype)
    w.psf_sigma = sigma
    return w


CASES = {
    "2d_s1.5": lambda: _case(51, (45, 53), 1.5),
    "2d_s4_ragged": lambda: _case(52, (37, 70), 4.0),
    "2d_two_labels": lambda: _case(53, (40, 40), 2.5, n_labels=2),
    "2d_four_labels": lambda: _case(54, (33, 47), 2.0, n_labels=4),
    "3d_s1": lambda: _case(55, (13, 15, 17), 1.0),
    "3d_u16_s1.5": lambda: _case(56, (12, 14, 11), 1.5, dtype=np.uint16, lam=30.0),
    "2d_wide_psf": lambda: _case(57, (24, 30), 16.0),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_deconv_gradients(ora, name):
    w = CASES[name]()
    print(f"[case {name} shape={w.image.shape} sigma={w.psf_sigma}]", flush=True)
    P = ora.params_of(w)
    ctx, img, lab = gpu_state(w)
    lin_o, a_o, b_o = ora.particles(P, w.labels)
    perm, lin, a, b = match_order(ctx, lin_o, b_o)
    dl2 = S.compute_l2_diff(ctx)
    o_l2 = ora.l2diff(P, w.image, w.labels, lin_o, a_o, b_o)
    assert rel_err(dl2[: len(lin)].cpu().numpy()[perm], o_l2) <= REL_GRAD
    dh1 = S.sobolev_smooth(ctx, dl2)[: len(lin)].cpu().numpy()[perm]
    assert rel_err(dh1, ora.sobolev(P, lin_o, a_o, b_o, o_l2)) <= REL_GRAD


@pytest.mark.parametrize("name", ["2d_s1.5", "3d_s1", "2d_two_labels"])
def test_deconv_trajectory(ora, name):
    """Eight iterations, each checked against the oracle stepping from the
    GPU's labels (gradients on every particle, labels outside the margin)."""
    w = CASES[name]()
    print(f"[case {name} trajectory]", flush=True)
    ctx, img, lab = gpu_state(w)
    sh = Shadow(ora, w, ctx).run(8)
    sh.report(name)
    assert sh.checked == 8


@pytest.mark.parametrize("tile", [S.TILE_DEFAULT, S.TILE_WIDE])
def test_deconv_full_size_first_steps(ora, tile):
    """The 512^2 scene with a sigma = 15 PSF, on the default cells and on the
    16x32 cells its benchmark's autotuner keeps: particle set, L2 and Sobolev
    gradients on every particle and the labels of the first three
    iterations, each checked from the GPU's labels."""
    w = W.make("deconv2d_512")
    w.tile = tile
    print(f"[case deconv2d_512 tile {tile}]", flush=True)
    ctx, img, lab = gpu_state(w)
    sh = Shadow(ora, w, ctx).run(3)
    sh.report("deconv2d_512")
    assert sh.checked == 3


def test_psf_contexts_are_not_batched():
    w = CASES["2d_s1.5"]()
    ctx, img, lab = gpu_state(w)
    batch = S.Batch(2)
    try:
        with pytest.raises(S.SobrcError) as e:
            batch.set(0, ctx)
        assert e.value.code == S.EINVAL
    finally:
        batch.close()


def test_deconv_with_topological_control(ora):
    """The deconvolving gradient driving the ranked, controlled acceptance:
    eight iterations, each checked against the oracle from the GPU's labels
    (a ranked decision is marginal near small or nearly tied gradients)."""
    from test_gpu_topology import topo_shadow_marginal
    w = _case(58, (36, 44), 2.0, n_labels=3, lam=0.2)
    w.topo = S.TOPO_SIMPLE
    print("[case deconv + topo]", flush=True)
    ctx, img, lab = gpu_state(w)
    sh = Shadow(ora, w, ctx, marginal=topo_shadow_marginal(w)).run(8)
    sh.report("deconv + topo")
    assert sh.checked == 8
