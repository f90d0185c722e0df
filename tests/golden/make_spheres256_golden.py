"""Write the expected values of the 256^3 mixed-form parity test.

The 256^3 random-sphere cell (spheres r ~ U[5, 15] to volume fraction 0.25,
contrast 10, E11 -> 0.01 over 20 steps, tolerance 1e-6) is taken through load
step 1 by the FP64 oracle on a fixed schedule of two loop iterations.  Stored
(spheres256_step1.npz): iters (1,), resp (1, 40) the step's averages, idx the
flat indices of the sampled voxels (4096 seeded random voxels, then the x row
and the z column through the centre of the first sphere), and the fields e,
g, t, m (9, K), p, q (K,) there.

Only the oracle and the seeded input generator are called.  It needs about
60 GB of host memory and a few minutes.  Run from the repository root:
    python tests/golden/make_spheres256_golden.py [out_dir]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import micropolar as O  # noqa: E402
from paper_2409_10774_amd import workloads as W  # noqa: E402

ITERS = 2


def main():
    out_dir = sys.argv[1] if len(sys.argv) > 1 else os.path.dirname(os.path.abspath(__file__))
    wl = W.random_spheres_256(n_steps=1)
    _, spheres = W.random_spheres(256, 2, None, 5.0, 15.0, target_vf=0.25)
    n = 256
    rng = np.random.default_rng(256)
    cx, cy, cz = (int(np.floor(v)) % n for v in spheres[0][:3])
    idx = np.concatenate([rng.choice(n ** 3, size=4096, replace=False),
                          (cz * n + cy) * n + np.arange(n),
                          (np.arange(n) * n + cy) * n + cx]).astype(np.int64)
    t0 = time.time()
    solver = O.Solver(wl.phase_map, wl.phases, h=wl.h, tol=wl.tol, norm=wl.err_norm,
                      ref_mode=wl.ref_mode)
    print(f"oracle set up in {time.time() - t0:.0f} s", flush=True)
    out = solver.solve(wl.times, wl.E, wl.G, schedule=[ITERS], fields_at=(1,))
    print(f"step 1: {ITERS} iterations, T11 {out['resp'][0][0]:.9e}, {time.time() - t0:.0f} s", flush=True)
    f = out["fields"][1]
    flat = {k: np.asarray(f[k]).reshape((9, -1) if k in "egtm" else (-1,)) for k in "egtmpq"}
    path = os.path.join(out_dir, "spheres256_step1.npz")
    np.savez(path, iters=np.array([ITERS]), resp=np.array(out["resp"]), idx=idx,
             **{k: (v[:, idx] if v.ndim == 2 else v[idx]) for k, v in flat.items()})
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
