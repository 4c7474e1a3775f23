"""Shadow-oracle checks of GPU iterations (helper of the GPU tests).

At every checked iteration the oracle takes one step from the GPU's own label
field, so a marginal decision never ends a comparison: the next iteration is
again compared from one shared state.  Bars:
  * particle sets: bit-exact (key = linear index, target label);
  * L2 and Sobolev gradients of the state: max |gpu - oracle| <= 1e-5 max |oracle|
    on every particle (fp32 against FP64);
  * labels after the step: identical at every pixel whose decision is not
    marginal (a particle with |g| <= 1e-4 max |g|, or two negative gradients
    of one pixel within that margin of each other); marginal differences are
    counted and returned;
  * flips and reversals the GPU reports: exactly those of its own label
    sequence; the flips equal the oracle's when no pixel differs;
  * region statistics: exact for the GPU's own new labels (uint16 sums
    exact, fp32 sums within 1e-6 of the largest).
"""
import os

import numpy as np
import torch

from paper_1403_0240_amd import sobrc as S

REL_GRAD = 1e-5
MARGIN = 1e-4


def oracle_threads():
    return max(1, min(os.cpu_count() or 1, 16))


def keys(lin, b):
    return np.asarray(lin, np.int64) * 65536 + np.asarray(b, np.int64)


def gpu_particles(ctx):
    lin, a, b = (t.cpu().numpy() for t in S.get_particles(ctx))
    return lin.astype(np.int64), a, b


def match_order(ctx, lin_o, b_o):
    """Permutation taking GPU (context) order to oracle order; asserts that
    the two particle sets are identical."""
    lin, a, b = gpu_particles(ctx)
    gk = keys(lin, b)
    perm = np.argsort(gk, kind="stable")
    ok = keys(lin_o, b_o)
    assert len(gk) == len(ok), f"particle count {len(gk)} != oracle {len(ok)}"
    assert np.array_equal(gk[perm], ok), "particle sets differ"
    return perm, lin, a, b


def rel_err(g, o):
    if len(o) == 0:
        return 0.0
    return float(np.abs(np.asarray(g, np.float64) - o).max() / max(np.abs(o).max(), 1e-300))


def marginal_pixels(lin, g, thr):
    """Pixels whose decision may depend on rounding: a particle with |g| <=
    thr, or two negative gradients of the pixel within thr of each other."""
    lin = np.asarray(lin, np.int64)
    g = np.asarray(g, np.float64)
    order = np.lexsort((g, lin))
    ls, gs = lin[order], g[order]
    close = (ls[1:] == ls[:-1]) & (gs[:-1] < 0) & (gs[1:] - gs[:-1] <= thr)
    return np.unique(np.concatenate([lin[np.abs(g) <= thr], ls[1:][close]]))


def compare_labels(L_gpu, L_ora, lin, g):
    """Labels agree at all non-marginal pixels; returns the number of
    (marginal) differing pixels."""
    thr = MARGIN * (np.abs(g).max() if len(g) else 1.0)
    diff = np.flatnonzero(L_gpu.reshape(-1) != L_ora.reshape(-1))
    if len(diff):
        bad = diff[~np.isin(diff, marginal_pixels(lin, g, thr))]
        assert len(bad) == 0, f"{len(bad)} non-marginal pixels differ, e.g. {bad[:5].tolist()}"
    return len(diff)


def check_stats(ora, P, w, ctx, L_gpu):
    n_g, s_g = S.get_region_stats(ctx)
    n_o, s1_o, _ = ora.region_stats(P, w.image, L_gpu)
    assert np.array_equal(n_g, n_o), "region pixel counts differ"
    if w.image.dtype == np.uint16:
        assert np.array_equal(s_g, s1_o), "region sums differ"
    else:
        assert np.allclose(s_g, s1_o, rtol=0, atol=1e-6 * max(1.0, np.abs(s1_o).max()))


def check_gradients(ora, ctx, info, perm, with_sobolev=True):
    n = len(perm)
    dl2 = S.compute_l2_diff(ctx)
    e2 = rel_err(dl2[:n].cpu().numpy()[perm], info["dE_l2"])
    assert e2 <= REL_GRAD, f"L2 gradient error {e2:.3g}"
    e1 = 0.0
    if with_sobolev:
        dh1 = S.sobolev_smooth(ctx, dl2)
        e1 = rel_err(dh1[:n].cpu().numpy()[perm], info["dE_h1"])
        assert e1 <= REL_GRAD, f"Sobolev gradient error {e1:.3g}"
    return e2, e1


class Shadow:
    """Runs a context step by step, each step checked against the oracle
    stepping from the GPU's labels.  mode: S.MODE_SOBOLEV / S.MODE_L2 /
    S.MODE_AUTO (the oracle's AUTO rule, fed with the GPU's own sequence,
    names each iteration's gradient and the stop); tol: flip tolerance of
    the run (AUTO and the tolerance stop)."""

    def __init__(self, ora, w, ctx, mode=S.MODE_SOBOLEV, tol=0.0, threads=None, marginal=None):
        self.ora, self.w, self.ctx = ora, w, ctx
        self.mode, self.tol = mode, tol
        self.P = ora.params_of(w, threads=threads or oracle_threads())
        self.rule = ora.AutoRule(mode, tol)
        self.stamp = np.zeros(w.labels.size, np.uint32)
        self.L = S.get_labels(ctx).cpu().numpy()
        self.marginal = marginal or (lambda info, g, L_g, L_o: compare_labels(L_g, L_o, info["lin"], g))
        self.steps = 0
        self.checked = 0
        self.marginal_flips = 0
        self.max_err = [0.0, 0.0]
        self.stopped = False
        self.nfl = torch.zeros(1, dtype=torch.int32, device=ctx.device)

    def pre(self, check=True, grads=True):
        """Checks of the state before an iteration; returns what post needs."""
        assert not self.stopped, "the run has stopped"
        ora, ctx = self.ora, self.ctx
        grad_mode = self.rule.grad
        L_o, info = None, None
        if check:
            L_o, info = ora.step(self.P, self.w.image, self.L, grad_mode)
            perm, _, _, _ = match_order(ctx, info["lin"], info["b"])
            if grads:
                e2, e1 = check_gradients(ora, ctx, info, perm, with_sobolev=grad_mode == ora.MODE_SOBOLEV)
                self.max_err = [max(self.max_err[0], e2), max(self.max_err[1], e1)]
        return grad_mode, S.particle_count(ctx), L_o, info

    def post(self, state):
        """Checks after the GPU ran the iteration; returns the number of
        marginal label differences (0 when not checked)."""
        grad_mode, n_t, L_o, info = state
        ora, w, ctx = self.ora, self.w, self.ctx
        L_g = S.get_labels(ctx).cpu().numpy()
        changed = L_g.reshape(-1) != self.L.reshape(-1)
        flips = int(changed.sum())
        back = ora.reversals(self.L.reshape(-1), L_g.reshape(-1), self.stamp, self.steps)
        hn, hf, hb = S.get_history(ctx, cap=1, reversals=True)
        assert (int(hn[-1]), int(hf[-1]), int(hb[-1])) == (n_t, flips, back), \
            f"iteration {self.steps}: GPU telemetry {(hn[-1], hf[-1], hb[-1])} != {(n_t, flips, back)}"
        nd = 0
        if info is not None:
            g = info["dE_h1"] if grad_mode == ora.MODE_SOBOLEV else info["dE_l2"]
            nd = self.marginal(info, g, L_g, L_o)
            if nd == 0:
                assert flips == info["flips"]
            check_stats(ora, self.P, w, ctx, L_g)
            self.checked += 1
            self.marginal_flips += nd
        self.stopped = self.rule.update(n_t, flips, back)
        if self.mode == S.MODE_AUTO:
            assert S.gradient_switch(ctx) == self.rule.switch_iter
        self.L = L_g
        self.steps += 1
        return nd

    def step(self, check=True, grads=True):
        """One iteration of the context on its own (checked against the oracle
        when check); returns the number of marginal label differences."""
        state = self.pre(check, grads)
        if self.mode == S.MODE_AUTO or self.tol > 0:
            assert S.run(self.ctx, 1, self.tol, self.mode) == 1
        else:
            S.step(self.ctx, self.mode, self.nfl)
        return self.post(state)

    def resume(self, mode, tol):
        """Continue after a stop with another plain mode (not AUTO) and
        tolerance; the reversal stamps carry on."""
        assert mode != S.MODE_AUTO
        self.mode, self.tol = mode, tol
        self.rule = self.ora.AutoRule(mode, tol)
        self.stopped = False
        return self

    def run(self, iters, check_at=None, grads=True):
        """Up to iters iterations or the stop; check_at: iterations (counted
        from this shadow's start) to check, None = all."""
        for _ in range(iters):
            if self.stopped:
                break
            self.step(check=check_at is None or self.steps in check_at, grads=grads)
        return self

    def report(self, name):
        print(f"  {name}: {self.steps} iterations, {self.checked} checked against the oracle, "
              f"{self.marginal_flips} marginal label differences, max rel. error "
              f"L2 {self.max_err[0]:.2e} Sobolev {self.max_err[1]:.2e}", flush=True)
