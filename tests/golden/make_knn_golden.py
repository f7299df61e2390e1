"""Writes tests/golden/knn_oracle_samples.npz: FP64 oracle K-NN results
(oracle/knn.py, Section II) for the two large point sets of the GPU tests.

  * latent: the 70000 points in a 3-D latent space behind the clustering
    workload's column graph; every row is computed (sigma needs all of
    them), and sigma plus 2000 sampled rows are stored;
  * digits: 70000 digit-shaped points of dimension 784; 500 sampled query
    rows are computed by brute force against all points.

K = 10 for both. Run: python tests/golden/make_knn_golden.py (single
process, a few minutes).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import knn as OK  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "knn_oracle_samples.npz")


def main():
    t0 = time.time()
    lat = synth.cluster_digits(0).meta["latent"]
    idx, d2 = OK.knn(lat, 10)
    sigma = OK.sigma_of(d2)
    rng = np.random.default_rng(77)
    lq = np.sort(rng.choice(lat.shape[0], size=2000, replace=False))
    print(f"latent: sigma {sigma:.15e}, {time.time() - t0:.1f} s", flush=True)
    pts, _ = synth.digits_points(0)
    dq = np.sort(rng.choice(pts.shape[0], size=500, replace=False))
    didx, dd2 = OK.query_knn(pts, dq, 10)
    print(f"digits: {time.time() - t0:.1f} s", flush=True)
    np.savez(OUT, lat_q=lq, lat_idx=idx[lq], lat_d2=d2[lq], lat_sigma=sigma,
             dig_q=dq, dig_idx=didx, dig_d2=dd2)
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
