"""sobolev_smooth_particles_static: the stateless Eq. (6) update with the
library's static scratch memory, through the C ABI, against the entry point
that takes a workspace and against the FP64 oracle, on two calls in a row
(the second with fewer particles on a smaller grid, so the scratch memory
holds the first call's contents), and its size limit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1403_0240_amd import sobrc as S  # noqa: E402
from paper_1403_0240_amd import workloads as W  # noqa: E402
from shadow import REL_GRAD, rel_err  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.lib()


def _particles(ora, seed, shape, n_labels, E):
    w = W.random_multilabel(seed, shape, n_labels, E=E)
    P = ora.params_of(w)
    lin, a, b = ora.particles(P, w.labels)
    perm = np.random.default_rng(seed).permutation(len(lin))  # any order
    lin, a, b = lin[perm], a[perm], b[perm]
    vals = np.random.default_rng(seed + 1).normal(size=len(lin)).astype(np.float32)
    p = S.make_params(shape, "float32", E, 0.0, max_labels=n_labels)
    dev = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in
           (lin.astype(np.int32), a.astype(np.int32), b.astype(np.int32), vals)]
    return P, p, (lin, a, b, vals), dev


def test_static_scratch_matches_workspace_entry_point(ora):
    cases = [(61, (23, 41, 37), 3, 6.0), (62, (90, 70), 3, 8.0)]  # 3D, then a smaller 2D call
    for seed, shape, M, E in cases:
        P, p, (lin, a, b, vals), (dl, da, db, dv) = _particles(ora, seed, shape, M, E)
        print(f"[static scratch: {len(lin)} particles, grid {shape}]", flush=True)
        out_s = torch.full((len(lin),), float("nan"), device="cuda")
        S.sobolev_smooth_particles_static(p, dl, da, db, dv, out_s)
        out_w = S.sobolev_smooth_particles(p, dl, da, db, dv)
        gs, gw = out_s.cpu().numpy(), out_w.cpu().numpy()
        o = ora.sobolev(P, lin, a, b, vals.astype(np.float64), neigh=ora.NEIGH_BRUTE)
        assert np.isfinite(gs).all()
        assert rel_err(gs, o) <= REL_GRAD
        assert rel_err(gs, gw) <= REL_GRAD
    # bad input is refused as by the workspace entry point
    with pytest.raises(S.SobrcError) as e:
        bad = torch.tensor([0, 10 ** 7], dtype=torch.int32, device="cuda")
        z = torch.zeros(2, dtype=torch.int32, device="cuda")
        S.sobolev_smooth_particles_static(p, bad, z, z + 1, torch.zeros(2, device="cuda"),
                                          torch.zeros(2, device="cuda"))
    assert e.value.code == S.EINVAL
