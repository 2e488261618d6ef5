"""Learned form of the step: a per-bond rank predictor sets the sketch widths
of the randomised rounding that replaces the deterministic truncations of
the RK4 sums (the stage inputs and the final combination), with the
deterministic QR + SVD rounding kept as the fallback whenever the a
posteriori error of the randomised result exceeds the tolerance (the
truncation of Sec. 2.3 / App. A.4 stays the reference).

The predictor is the device MLP (``tt.MLP``: FP16 parameters, FP32
accumulation, trained by the library's own forward/backward/Adam kernels).
Per interior bond k of a step it reads what the previous step's final
rounding reported and returns the rank that this step's rounding will keep:

    inputs   r_k / rmax, the last 8 kept singular values of bond k relative
             to the norm (log10, divided by 10, floored at 1e-20), log10(nu),
             the time t, the bond position k / d, and log10(norm) / d;
    target   the rank the deterministic final rounding keeps at bond k in
             the next step, divided by rmax.

Training data come from trajectories of the plain solver (deterministic
rounding), one sample per interior bond and step.  The widths handed to the
step are the predicted ranks plus ``OVERSAMPLE``; when a predicted rank
reaches the cap the rounding is cap-limited, the randomised result cannot
meet a tolerance that the deterministic rounding itself misses, and the step
runs without the learned widths.

The stage applications' sketch widths follow the ranks the previous step's
rounded stage derivatives kept (plus the same oversampling); a stage whose
rounded derivative reaches its width at some bond is applied again at the
plain width.
"""
import math
import time

import numpy as np

from . import tt

N_FEATURES = 13
OVERSAMPLE = 8
SV_FLOOR = 1e-20
WIDTH = 128


def bond_features(ranks, final_sv, final_norm, nu, t, rmax):
    """Features of the d-1 interior bonds from one step's report.

    ``ranks`` (d+1 ints), ``final_sv`` (d-1 lists of the 8 smallest kept
    singular values, decreasing, zeros in front when fewer were kept) and
    ``final_norm`` are the ``ranks``, ``final_sv`` and ``final_norm`` entries
    of ``tt.tt_step``'s report.  Returns float32 (d-1, N_FEATURES)."""
    d = len(ranks) - 1
    x = np.zeros((max(d - 1, 0), N_FEATURES), dtype=np.float32)
    norm = float(final_norm) if final_norm > 0 else 1.0
    lognorm = math.log10(norm) / d
    for k in range(1, d):
        sv = np.asarray(final_sv[k - 1], dtype=np.float64) / norm
        x[k - 1, 0] = ranks[k] / rmax
        x[k - 1, 1:9] = np.log10(np.maximum(sv, SV_FLOOR)) / 10.0
        x[k - 1, 9] = math.log10(nu)
        x[k - 1, 10] = t
        x[k - 1, 11] = k / d
        x[k - 1, 12] = lognorm
    return x


def widths_from_ranks(pred, d, rmax, oversample=OVERSAMPLE):
    """Sketch widths (d+1 ints) from predicted interior ranks, or None when
    a predicted rank reaches the cap (cap-limited rounding)."""
    pred = np.asarray(pred)
    if pred.size == 0 or int(pred.max()) >= rmax:
        return None
    return [1] + [int(min(512, max(1, p) + oversample)) for p in pred] + [1]


def apply_widths(k_ranks, rmax, sketch_rank, oversample=OVERSAMPLE):
    """Sketch widths of the stage applications from the ranks the previous
    step's rounded stage derivatives kept, or None when a bond reached the
    cap there (a cap-limited derivative gives no bound on the width)."""
    inner = [int(r) for r in k_ranks[1:-1]]
    if not inner or max(inner) >= rmax:
        return None
    return [1] + [min(sketch_rank, max(1, r) + oversample) for r in inner] + [1]


def he_init(n_in, width, seed):
    """He-uniform weights, zero biases, in the MLP's parameter order."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, shape in ((n_in, (width, n_in)), (width, (width, width)), (width, (1, width))):
        lim = math.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, size=shape).ravel())
        parts.append(np.zeros(shape[0]))
    return np.concatenate(parts).astype(np.float32)


class RankPredictor:
    """The trained network and the rank/width rule around it."""

    def __init__(self, ctx, rmax, max_batch=16384, width=WIDTH, seed=0):
        self.ctx, self.rmax = ctx, rmax
        self.net = tt.MLP(ctx, N_FEATURES, width, max_batch)
        self.net.set_params(he_init(N_FEATURES, width, seed))
        self.max_batch = max_batch

    def fit(self, x, ranks_next, iters=3000, lr=2e-3):
        """Full-batch Adam on (features, next ranks / rmax); returns the
        loss before and after."""
        import torch

        if x.shape[0] > self.max_batch:
            raise ValueError("more samples than the network's batch capacity")
        xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
        td = torch.from_numpy(np.ascontiguousarray(ranks_next, dtype=np.float32) / self.rmax).cuda()
        l0, _ = self.net.gradients(xd, td)
        l1 = self.net.train(xd, td, iters, lr)
        return l0, l1

    def predict(self, x):
        """Predicted ranks (ints in 1..rmax) for a feature matrix."""
        import torch

        xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
        y = self.net.forward(xd).cpu().numpy()
        return np.clip(np.rint(y * self.rmax), 1, self.rmax).astype(np.int64)

    def close(self):
        self.net.close()


def run_trajectory(ctx, op, f, steps, dt, rmax, eps, sketch_rank, nu, predictor=None, tol=1e-6, seed=0,
                   precision=0, on_step=None):
    """``steps`` RK4 steps of f in place (sketched apply), the plain form
    when ``predictor`` is None, else the learned form (widths predicted
    from the previous step's report; the first step is plain).  Returns a
    list of per-step records: wall time (prediction included), ranks,
    learned_used / learned_fallback / learned_err, and the features of the
    step's report (for data capture)."""
    recs = []
    rep = None
    t = 0.0
    for s in range(steps):
        ctx.sync()
        t0 = time.perf_counter()
        widths = awidths = None
        if predictor is not None and rep is not None:
            feats = bond_features(rep["ranks"], rep["final_sv"], rep["final_norm"], nu, t, rmax)
            widths = widths_from_ranks(predictor.predict(feats), f.d, rmax)
            awidths = apply_widths(rep["k_ranks"], rmax, sketch_rank) if widths is not None else None
        rep = tt.tt_step(ctx, op, f, dt, rmax, eps, tt.TT_APPLY_SKETCH, sketch_rank, seed + s, precision=precision,
                         learned_widths=widths, learned_tol=tol, learned_apply_widths=awidths)
        ctx.sync()
        wall = time.perf_counter() - t0
        t += dt
        rec = {"wall": wall, "ranks": rep["ranks"], "widths": widths, "learned_used": rep["learned_used"],
               "learned_fallback": rep["learned_fallback"], "learned_err": rep["learned_err"],
               "apply_widths": awidths, "apply_fallback": rep["learned_apply_fallback"],
               "features": bond_features(rep["ranks"], rep["final_sv"], rep["final_norm"], nu, t, rmax)}
        recs.append(rec)
        if on_step is not None:
            on_step(s, rec)
    return recs


def samples_from_records(recs):
    """Training pairs from one plain trajectory: the features of step s's
    report and the interior ranks of step s+1."""
    xs, ys = [], []
    for a, b in zip(recs[:-1], recs[1:]):
        xs.append(a["features"])
        ys.append(np.asarray(b["ranks"][1:-1], dtype=np.float32))
    if not xs:
        return np.zeros((0, N_FEATURES), np.float32), np.zeros(0, np.float32)
    return np.concatenate(xs), np.concatenate(ys)
