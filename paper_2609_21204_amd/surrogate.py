"""Learned surrogate of the parameter sweep.

A 4 -> 128 -> 128 -> 2 perceptron (kernels in csrc/mlp.hip) maps a sweep
point -- bond free energy eps (in kT), number density rho, crosslinker
valence cap_B (A sites have valence 1) and temperature kT -- to the two
observables a sweep is run for: the bonded fraction of the A-B reaction and
the largest-cluster fraction (largest connected component of static plus
dynamic bonds over N).  Both are averages over the last quarter of runs of
replicas simulated by the library itself (db_step_batch), so the network
learns what the simulator produces.

The network then picks where the next plain simulations are spent: a large
uniform pool of candidate points is scored and the points predicted closest
to a target value (by default the percolation line, largest-cluster fraction
0.5) are simulated with db_step, one replica after another.  Each plain run
judges its prediction; where the two differ by more than the tolerance
(0.02) the plain value is kept (fallback), otherwise the prediction stands.

Replica size N and kind (monomers or telechelic chains) are not inputs: N
is drawn log-uniform per replica, and one network is trained per kind.
"""

import dataclasses
import math
import time

import numpy as np

from . import dybond as db
from . import inputs

# sweep ranges (eps, rho and cap_B as in the replica generator; kT added so
# that the fourth input varies)
EPS = (2.0, 10.0)
RHO = (0.05, 0.4)
CAPS = (1, 2, 4)
KT = (0.8, 1.2)
N_RANGE = (256, 8192)
TOLERANCE = 0.02
OUTPUTS = ("bonded_fraction", "largest_cluster_fraction")


@dataclasses.dataclass
class Points:
    """A set of sweep points (one entry per replica)."""
    eps: np.ndarray
    rho: np.ndarray
    cap_b: np.ndarray
    kT: np.ndarray
    n: np.ndarray
    seed: np.ndarray
    kind: str

    def __len__(self):
        return len(self.eps)

    def take(self, idx):
        idx = np.asarray(idx)
        return Points(self.eps[idx], self.rho[idx], self.cap_b[idx], self.kT[idx], self.n[idx], self.seed[idx],
                      self.kind)

    def features(self):
        """Network inputs, each mapped onto [-1, 1]."""
        return np.stack([(self.eps - 0.5 * (EPS[0] + EPS[1])) / (0.5 * (EPS[1] - EPS[0])),
                         (self.rho - 0.5 * (RHO[0] + RHO[1])) / (0.5 * (RHO[1] - RHO[0])),
                         np.log2(self.cap_b) - 1.0,
                         (self.kT - 0.5 * (KT[0] + KT[1])) / (0.5 * (KT[1] - KT[0]))],
                        axis=1).astype(np.float32)


def draw_points(rng, count, kind, n_range=N_RANGE, seed_base=0):
    """Uniform sweep points: eps, rho, kT uniform, cap_B uniform over
    {1, 2, 4}, N log-uniform; replica seeds seed_base + k."""
    n = np.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1]), count)).astype(np.int64)
    return Points(eps=rng.uniform(*EPS, count), rho=rng.uniform(*RHO, count),
                  cap_b=rng.choice(np.array(CAPS), count), kT=rng.uniform(*KT, count), n=n,
                  seed=seed_base + np.arange(count, dtype=np.int64), kind=kind)


def _workload(p, k):
    return inputs.replica(int(p.seed[k]), int(p.n[k]), float(p.eps[k]), float(p.rho[k]), int(p.cap_b[k]),
                          p.kind, kT=float(p.kT[k]))


SEED_STRIDE = 100_003     # replica seeds of one point: seed, seed + stride, ...


def replicas_of(points, seeds):
    """Each point repeated `seeds` times with seeds seed + j * SEED_STRIDE
    (same parameters and N, other initial state and noise); replica
    j * len(points) + k is seed j of point k."""
    if seeds == 1:
        return points
    idx = np.tile(np.arange(len(points)), seeds)
    rep = points.take(idx)
    rep.seed = rep.seed + np.repeat(np.arange(seeds, dtype=np.int64), len(points)) * SEED_STRIDE
    return rep


def simulate(points, steps=20000, samples=5, plain=False, chunk=1024, device=0, log=None, seeds=1):
    """Observables of every point: (len(points), 2) end-of-run averages of
    (bonded fraction, largest-cluster fraction) over `samples` equally spaced
    reads in the last quarter of a `steps`-step run, averaged over `seeds`
    replicas of the point (replicas_of), which run in the same batches.

    plain=False runs each chunk of replicas together (db_step_batch);
    plain=True runs every replica on its own with db_step.  Both give the
    same trajectory bit for bit, so they differ only in time."""
    if seeds > 1:
        per = simulate(replicas_of(points, seeds), steps, samples, plain, chunk, device, log)
        return per.reshape(seeds, len(points), 2).mean(axis=0)
    span = (steps // 4) // samples
    if span < 1:
        raise ValueError("steps must be at least 4 * samples")
    first = steps - span * samples
    out = np.zeros((len(points), 2))
    for c0 in range(0, len(points), chunk):
        idx = range(c0, min(len(points), c0 + chunk))
        systems = [db.System.from_workload(_workload(points, k), device) for k in idx]
        try:
            if plain:
                for s, k in zip(systems, idx):
                    s.step(first)
                    for _ in range(samples):
                        s.step(span)
                        o = s.observables()
                        out[k] += (o["bonded_fraction"][0], o["largest_cluster_fraction"])
            else:
                hs = [s.h for s in systems]
                db.db_step_batch(hs, first)
                for _ in range(samples):
                    db.db_step_batch(hs, span)
                    for s, k in zip(systems, idx):
                        o = s.observables()
                        out[k] += (o["bonded_fraction"][0], o["largest_cluster_fraction"])
        finally:
            for s in systems:
                s.close()
        if log:
            log(f"simulated {idx.stop}/{len(points)} {points.kind} replicas")
    return out / samples


def init_params(seed):
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases, in the flat
    order W1 (128 x 4), b1, W2 (128 x 128), b2, W3 (2 x 128), b3."""
    rng = np.random.default_rng(seed)
    parts = []
    for rows, cols in ((128, 4), (128, 128), (2, 128)):
        bound = math.sqrt(6.0 / cols)
        parts += [rng.uniform(-bound, bound, rows * cols), np.zeros(rows)]
    flat = np.concatenate(parts).astype(np.float32)
    assert flat.size == db.MLP_PARAMS
    return flat


class Surrogate:
    """One network on the GPU (owns a db_mlp handle)."""

    def __init__(self, seed=0, batch_max=1024, device=0):
        self.h = db.db_mlp_create(batch_max, device)
        db.db_mlp_set_params(self.h, init_params(seed))
        self.batch_max = batch_max

    def close(self):
        if self.h:
            db.db_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def fit(self, points, targets, epochs=400, batch=256, lr=(3e-3, 1e-3, 3e-4, 1e-4), seed=0):
        """Adam on the mean-squared error, the epochs split evenly over the
        learning rates in `lr` (a step-down schedule); returns the final
        training loss."""
        x = points.features()
        t = np.asarray(targets, dtype=np.float32)
        loss = float("nan")
        per = max(1, epochs // len(lr))
        for k, rate in enumerate(lr):
            loss = db.db_mlp_train(self.h, x, t, batch=min(batch, self.batch_max), epochs=per, lr=rate,
                                   seed=seed * 1000 + k)
        return loss

    def predict(self, points):
        return db.db_mlp_predict(self.h, points.features()).astype(np.float64)

    def params(self):
        return db.db_mlp_get_params(self.h)


def choose(model, rng, count, kind, target=0.5, output=1, pool=65536, n_range=N_RANGE, seed_base=0):
    """The `count` points of a uniform candidate pool whose predicted
    `output` lies closest to `target`; replica seeds seed_base + k."""
    cand = draw_points(rng, pool, kind, n_range)
    pred = model.predict(cand)[:, output]
    best = np.argsort(np.abs(pred - target), kind="stable")[:count]
    chosen = cand.take(best)
    chosen.seed = seed_base + np.arange(count, dtype=np.int64)
    return chosen


def judge(pred, plain, tol=TOLERANCE):
    """Per-point verdict of the predictions against plain runs: the value
    kept (prediction where every output is within tol, else the plain run),
    the fallback mask and the absolute errors."""
    err = np.abs(np.asarray(pred) - np.asarray(plain))
    fallback = np.any(err > tol, axis=1)
    kept = np.where(fallback[:, None], plain, pred)
    return kept, fallback, err


def hit_rate(values, target=0.5, band=0.1):
    """Fraction of points whose value lies within band of target."""
    return float(np.mean(np.abs(np.asarray(values) - target) <= band))


def run_workflow(train_replicas=20480, steps=20000, samples=5, points=256, kinds=("chains", "mono"),
                 n_range=N_RANGE, epochs=400, batch=256, pool=65536, uniform_plain=True, seed=1, device=0,
                 log=print, seeds=4, judge_batched=True):
    """Train one network per kind on simulated replicas (equal shares of
    train_replicas, `seeds` replicas per sweep point averaged into its label,
    one point in ten held out), then let the first kind's network choose
    `points` new points near the percolation line and judge each by the
    simulation (the same `seeds` replicas per point, batched when
    judge_batched: batched runs equal db_step runs bit for bit, so this is
    the plain method, only faster).  A second, disjoint set of `seeds`
    replicas of the chosen points gives the noise floor of a label: the
    spread of two such averages, over sqrt(2) for one of them.  The uniform
    sweep the chosen points are compared with is `points` uniform points run
    the same way (uniform_plain) or else the uniform training points."""
    rng = np.random.default_rng(seed)
    report = {"train_replicas": train_replicas, "seeds_per_point": seeds, "steps": steps, "samples": samples,
              "points": points, "n_range": list(n_range), "epochs": epochs}
    plain_run = not judge_batched
    nets = {}
    uniform_lc = None
    try:
        for ki, kind in enumerate(kinds):
            count = train_replicas // len(kinds) // seeds
            pts = draw_points(rng, count, kind, n_range, seed_base=(seed * 10 + ki) * 1_000_000)
            t0 = time.perf_counter()
            tgt = simulate(pts, steps, samples, device=device, log=log, seeds=seeds)
            t_sim = time.perf_counter() - t0
            hold = np.arange(count) % 10 == 0
            net = Surrogate(seed=seed + ki, device=device)
            nets[kind] = net
            t0 = time.perf_counter()
            loss = net.fit(pts.take(~hold), tgt[~hold], epochs=epochs, batch=batch, seed=seed)
            t_fit = time.perf_counter() - t0
            err = np.abs(net.predict(pts.take(hold)) - tgt[hold])
            report[kind] = {"points": count, "replicas": count * seeds, "simulate_s": t_sim, "train_s": t_fit,
                            "train_loss": loss,
                            "heldout_mae": err.mean(axis=0).tolist(),
                            "heldout_within_tol": np.mean(err <= TOLERANCE, axis=0).tolist(),
                            "uniform_hit_rate": hit_rate(tgt[:, 1])}
            if ki == 0:
                uniform_lc = tgt[:, 1]
            log(f"{kind}: {report[kind]}")
        kind = kinds[0]
        chosen = choose(nets[kind], rng, points, kind, pool=pool, n_range=n_range,
                        seed_base=(seed * 10 + 7) * 1_000_000)
        pred = nets[kind].predict(chosen)
        t0 = time.perf_counter()
        plain = simulate(chosen, steps, samples, plain=plain_run, device=device, seeds=seeds)
        t_judge = time.perf_counter() - t0
        kept, fallback, err = judge(pred, plain)
        # the same points again with a disjoint set of seeds: how far two
        # `seeds`-replica averages of one point fall apart is what remains of
        # the replica noise in a label (and bounds how close any prediction
        # from these four inputs can come to one)
        again = chosen.take(np.arange(len(chosen)))
        again.seed = again.seed + 500_000
        spread = np.abs(simulate(again, steps, samples, device=device, seeds=seeds) - plain)
        if uniform_plain:
            uni = draw_points(rng, points, kind, n_range, seed_base=(seed * 10 + 8) * 1_000_000)
            uniform_lc = simulate(uni, steps, samples, plain=plain_run, device=device, seeds=seeds)[:, 1]
        h_c, h_u = hit_rate(plain[:, 1]), hit_rate(uniform_lc)
        report["chosen"] = {"kind": kind, "judge_s": t_judge,
                            "judged_by": "db_step_batch runs (bitwise equal to db_step)" if judge_batched
                            else "db_step runs, one replica after another",
                            "mae": err.mean(axis=0).tolist(),
                            "within_tol": np.mean(err <= TOLERANCE, axis=0).tolist(),
                            "fallbacks": int(fallback.sum()), "replica_spread": spread.mean(axis=0).tolist(),
                            "noise_floor": (spread.mean(axis=0) / math.sqrt(2.0)).tolist(),
                            "replica_spread_within_tol": np.mean(spread <= TOLERANCE, axis=0).tolist(),
                            "hit_rate_chosen": h_c, "hit_rate_uniform": h_u,
                            "uniform_source": "simulated uniform points" if uniform_plain else "training points",
                            "plain_runs_saved": 1.0 - h_u / h_c if h_c > 0 else 0.0}
        report["_arrays"] = {"pred": pred, "plain": plain, "kept": kept, "fallback": fallback}
        log(f"chosen: { {k: v for k, v in report['chosen'].items()} }")
    finally:
        for net in nets.values():
            net.close()
    return report


if __name__ == "__main__":
    import argparse
    import json

    ap = argparse.ArgumentParser(description="train the sweep surrogate and judge its chosen points")
    ap.add_argument("--train-replicas", type=int, default=20480)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--samples", type=int, default=5)
    ap.add_argument("--points", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=400)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--seeds", type=int, default=4, help="replicas averaged per sweep point")
    ap.add_argument("--plain-judge", action="store_true",
                    help="judge with db_step runs one replica after another (same numbers, slower)")
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    rep = run_workflow(a.train_replicas, a.steps, a.samples, a.points, epochs=a.epochs, seed=a.seed,
                       log=lambda m: print(m, flush=True), seeds=a.seeds, judge_batched=not a.plain_judge)
    rep.pop("_arrays")
    line = json.dumps(rep)
    print(line)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")
