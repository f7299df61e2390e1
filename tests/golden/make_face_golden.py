"""Writes tests/golden/face_oracle_samples.npz: the FP64 oracle's result on
the full face-shaped workload (p = 112 * 92 pixels, n = 1000 samples, rank
10, 10% outliers, 10% row/column sampling, gamma_r = gamma_c = 1), sampled
at fixed positions.

Pipeline (oracle only): FISTA for FRPCAG, 500 iterations (Algorithm 1), then
the alternate decoder (Section V.B) by textbook CG to a relative residual of
1e-13. Stored: a fingerprint of the inputs, 20000 sampled entries of the
FISTA output X~ and of X, both Frobenius norms, the oracle's CG iteration
count, its final residual and its condition-number estimate.

Run: python tests/golden/make_face_golden.py   (single-threaded, tens of
minutes of CPU time).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import decoder as OD  # noqa: E402
from oracle import frpcag as OF  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "face_oracle_samples.npz")


def fingerprint(P):
    rng = np.random.default_rng(321)
    pos = rng.choice(P.Ytil.size, size=64, replace=False)
    return np.concatenate([P.Ytil.ravel()[pos], P.Lr.data[:32], P.Lc.data[:32],
                           P.Lr_til.data[:32], P.Lc_til.data[:32],
                           [P.lmax_r_til, P.lmax_c_til, P.Ytil.sum()]])


def main():
    t0 = time.time()
    P = synth.cfg2_face(0)
    print(f"inputs: {time.time() - t0:.1f} s", flush=True)
    Xt, _ = OF.fista(P.Ytil, P.Lr_til, P.Lc_til, P.gamma_r, P.gamma_c, P.lmax_r_til,
                     P.lmax_c_til, 500)
    print(f"fista: {time.time() - t0:.1f} s", flush=True)
    m_r, m_c = OD.masks(P.p, P.n, P.omega_r, P.omega_c)
    B = OD.rhs(Xt, P.p, P.n, P.omega_r, P.omega_c)
    X, info = OD.solve_cg(B, m_r, m_c, P.Lr, P.Lc, P.gamma_r, P.gamma_c, tol=1e-13,
                          return_info=True)
    kappa = OD.cg_kappa_estimate(info["alphas"], info["betas"])
    print(f"cg: {info['iters']} it, rel.res {info['rel_residual']:.2e}, kappa {kappa:.3e}, "
          f"{time.time() - t0:.1f} s", flush=True)
    rng = np.random.default_rng(2025)
    idx_t = rng.choice(Xt.size, size=20000, replace=False)
    idx = rng.choice(P.p * P.n, size=20000, replace=False)
    np.savez(OUT, fingerprint=fingerprint(P), idx_t=idx_t, vals_t=Xt.ravel()[idx_t],
             Xtil_norm=np.linalg.norm(Xt), idx=idx, vals=X.ravel()[idx],
             norm=np.linalg.norm(X), iters=info["iters"], rel_residual=info["rel_residual"],
             kappa=kappa)
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
