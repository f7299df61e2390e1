"""Writes tests/golden/batch_oracle_samples.npz: FP64 oracle results for a
seeded subset of the batched workload (64 instances, p log-uniform in
[500, 4000], n log-uniform in [200, 2000], each on a 4 x 4 gamma grid).

The subset (TASKS) holds the largest instance at gamma = (100, 100) and
(0.1, 100), the ill-conditioned instance 5 at (0.1, 100), instance 7 at
(100, 0.1), and four tasks drawn with a seeded generator. Per task the
pipeline is the batched solve's, in the oracle: FISTA for FRPCAG, 100
iterations (Algorithm 1) on the FP32-rounded sampled matrix (the batched
inputs are FP32), the estimate rounded to FP32 (the batched solver hands
its FP32 estimate to the decoder), then the alternate decoder (Section V.B)
by textbook CG to a relative residual of 1e-13. Stored per task: 4000 sampled
entries of X, ||X||_F, the CG iteration count, the final residual and the
condition-number estimate, plus an input fingerprint per instance.

Run: python tests/golden/make_batch_golden.py --task T   (one task per
process, writes tests/golden/batch_parts/task_T.npz), then
python tests/golden/make_batch_golden.py --combine.
"""
import argparse
import glob
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import decoder as OD  # noqa: E402
from oracle import frpcag as OF  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "batch_oracle_samples.npz")
PARTS = os.path.join(HERE, "batch_parts")
FISTA_ITERS = 100
SAMPLES = 4000


def subset(probs):
    """(instance, gamma_r, gamma_c) of the checked tasks."""
    big = max(range(len(probs)), key=lambda k: probs[k].p * probs[k].n)
    tasks = [(big, 100.0, 100.0), (big, 0.1, 100.0), (5, 0.1, 100.0), (7, 100.0, 0.1)]
    rng = np.random.default_rng(11)
    vals = (0.1, 1.0, 10.0, 100.0)
    while len(tasks) < 8:
        t = (int(rng.integers(0, len(probs))), float(rng.choice(vals)), float(rng.choice(vals)))
        if t not in tasks:
            tasks.append(t)
    return tasks


def fingerprint(P):
    rng = np.random.default_rng(99)
    pos = rng.choice(P.Ytil.size, size=32, replace=False)
    return np.concatenate([P.Ytil.ravel()[pos], P.Lr.data[:16], P.Lc.data[:16],
                           P.Lr_til.data[:16], P.Lc_til.data[:16],
                           [P.lmax_r_til, P.lmax_c_til, P.p, P.n]])


def solve_task(P, gr, gc):
    Y = P.Ytil.astype(np.float32).astype(np.float64)
    Xt, _ = OF.fista(Y, P.Lr_til, P.Lc_til, gr, gc, P.lmax_r_til, P.lmax_c_til, FISTA_ITERS)
    Xt = Xt.astype(np.float32).astype(np.float64)
    m_r, m_c = OD.masks(P.p, P.n, P.omega_r, P.omega_c)
    B = OD.rhs(Xt, P.p, P.n, P.omega_r, P.omega_c)
    X, info = OD.solve_cg(B, m_r, m_c, P.Lr, P.Lc, gr, gc, tol=1e-13, max_iter=2000000,
                          return_info=True)
    kappa = OD.cg_kappa_estimate(info["alphas"], info["betas"])
    return X, info, kappa


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--task", type=int, default=None)
    ap.add_argument("--combine", action="store_true")
    args = ap.parse_args()
    t0 = time.time()
    probs, _ = synth.cfg5_batch(0)
    tasks = subset(probs)
    if args.combine:
        out = dict(tasks=np.array(tasks, dtype=np.float64))
        for t, (k, gr, gc) in enumerate(tasks):
            d = np.load(os.path.join(PARTS, f"task_{t}.npz"))
            for key in d.files:
                out[f"t{t}_{key}"] = d[key]
        np.savez(OUT, **out)
        for f in glob.glob(os.path.join(PARTS, "task_*.npz")):
            os.remove(f)
        os.rmdir(PARTS)
        print(f"wrote {OUT}", flush=True)
        return
    k, gr, gc = tasks[args.task]
    P = probs[k]
    print(f"task {args.task}: instance {k} ({P.p} x {P.n}), gamma ({gr}, {gc}); "
          f"inputs {time.time() - t0:.1f} s", flush=True)
    X, info, kappa = solve_task(P, gr, gc)
    print(f"task {args.task}: cg {info['iters']} it, rel.res {info['rel_residual']:.2e}, "
          f"kappa {kappa:.3e}, {time.time() - t0:.1f} s", flush=True)
    rng = np.random.default_rng(1000 + args.task)
    idx = rng.choice(P.p * P.n, size=SAMPLES, replace=False)
    os.makedirs(PARTS, exist_ok=True)
    np.savez(os.path.join(PARTS, f"task_{args.task}.npz"), fingerprint=fingerprint(P), idx=idx,
             vals=X.ravel()[idx], norm=np.linalg.norm(X), iters=info["iters"],
             rel_residual=info["rel_residual"], kappa=kappa)


if __name__ == "__main__":
    main()
