"""Write the expected values of the augmented-Lagrangian parity test on a
64^3 RVE at contrast 20.

The cell is the one of tests/test_gpu_al.py (contrast20_rve): a 64^3 RVE of
the many-RVE kind (random_rve seed 7: 57 spheres, volume fraction 0.115) with
the inclusion's moduli 20x the matrix's, tolerance 1e-6, its strain path
scaled 5x (norm 0.0025 at step 2, so that the matrix yields).  The oracle's
augmented-Lagrangian scheme (geometric-mean penalty, over-relaxation 1.7)
runs its first two load steps on a fixed schedule of 3 iterations each,
which crosses the scheme's first iterate, local steps on yielding voxels,
the commit and the extrapolated start of step 2.  Stored (al64_steps2.npz):
  iters  (2,)      the schedule
  resp   (2, 40)   volume averages per step: <t>, <m>, <e>, <gamma>, <p>,
                   <q>, <t_eq>, <m_eq>
  idx    (K,)      flat voxel indices (z n1 + y) n0 + x of the sampled voxels:
                   4096 seeded random voxels, then the x row through the cell's
                   centre
  e, g, t, m (9, K), p, q (K,)   the state after step 2 at those voxels

Only the oracle and the seeded input generator are called.  About four
minutes of one CPU core.  Run from the repository root:
    python tests/golden/make_al64_golden.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import augmented as AL  # noqa: E402
from tests.test_gpu_al import contrast20_rve  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "al64_steps2.npz")
SCHEDULE = [3, 3]
LOAD_SCALE = 5.0


def main():
    n = 64
    wl = contrast20_rve(n, len(SCHEDULE))
    wl.E = wl.E * LOAD_SCALE
    rng = np.random.default_rng(64)
    idx = np.concatenate([rng.choice(n ** 3, size=4096, replace=False),
                          ((n // 2) * n + n // 2) * n + np.arange(n)]).astype(np.int64)
    t0 = time.time()
    out = AL.ALSolver(wl.phase_map, wl.phases, tol=wl.tol, ref_mode="geometric_mean", relax=1.7).solve(
        wl.times, wl.E, wl.G, schedule=SCHEDULE, fields_at=(len(SCHEDULE),))
    print(f"oracle: {time.time() - t0:.0f} s, p max {out['resp'][:, 36].max():.3e}", flush=True)
    f = out["fields"][len(SCHEDULE)]
    flat = {k: np.asarray(f[k]).reshape((9, -1) if k in "egtm" else (-1,)) for k in "egtmpq"}
    np.savez(OUT, iters=np.array(SCHEDULE), resp=np.asarray(out["resp"]), idx=idx,
             **{k: (v[:, idx] if v.ndim == 2 else v[idx]) for k, v in flat.items()})
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
