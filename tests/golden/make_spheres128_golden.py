"""Write the expected values of the full-size parity test on the 128^3 cell.

The 128^3 random-sphere cell (40 elastic spheres r ~ U[6, 12], contrast 10,
E11 -> 0.02 and Gamma12 -> 0.002 over 50 steps, tolerance 1e-8, Eq. 38) is
solved by the FP64 oracle over its first three load steps, converged on the
oracle's own schedule.  Stored (spheres128_steps3.npz):
  iters  (3,)      loop iterations per step (Alg. 2)
  err    (3,)      error measure at the end of each step (Eqs. 36-38)
  resp   (3, 40)   volume averages per step: <t>, <m>, <e>, <gamma>, <p>,
                   <q>, <t_eq>, <m_eq>
  idx    (K,)      flat voxel indices (z n1 + y) n0 + x of the sampled voxels:
                   4096 seeded random voxels, then the x row and the z column
                   through the centre of the cell's first sphere
  e, g, t, m (9, K), p, q (K,)   the state after step 3 at those voxels

Only the oracle and the seeded input generator are called.  About an hour of
one CPU core.  Run from the repository root:
    python tests/golden/make_spheres128_golden.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import micropolar as O  # noqa: E402
from paper_2409_10774_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "spheres128_steps3.npz")


def sample_indices(n, sphere):
    """Seeded random voxels plus the x row and z column through a sphere centre."""
    rng = np.random.default_rng(128)
    nvox = n ** 3
    rand = rng.choice(nvox, size=4096, replace=False)
    cx, cy, cz = (int(np.floor(v)) % n for v in sphere[:3])
    row = (cz * n + cy) * n + np.arange(n)
    col = (np.arange(n) * n + cy) * n + cx
    return np.concatenate([rand, row, col]).astype(np.int64)


def main():
    wl = W.random_spheres_128(n_steps=3)
    _, spheres = W.random_spheres(128, 1, 40, 6.0, 12.0)
    idx = sample_indices(128, spheres[0])
    t0 = time.time()
    solver = O.Solver(wl.phase_map, wl.phases, h=wl.h, tol=wl.tol, norm=wl.err_norm,
                      ref_mode=wl.ref_mode)
    print(f"oracle set up in {time.time() - t0:.1f} s", flush=True)
    iters, errs, resp = [], [], []
    for s in range(1, 4):
        t1 = time.time()
        out = solver.solve(wl.times[s - 1: s + 1], wl.E[s - 1: s], wl.G[s - 1: s],
                           fields_at=(1,) if s == 3 else ())
        iters.append(out["iters"][0])
        errs.append(out["err"][0])
        resp.append(out["resp"][0])
        print(f"step {s}: {out['iters'][0]} iterations, err {out['err'][0]:.3e}, "
              f"T11 {out['resp'][0][0]:.9e}, {time.time() - t1:.0f} s", flush=True)
    f = out["fields"][1]
    flat = {k: np.asarray(f[k]).reshape((9, -1) if k in "egtm" else (-1,)) for k in "egtmpq"}
    np.savez(OUT, iters=np.array(iters), err=np.array(errs), resp=np.array(resp), idx=idx,
             **{k: (v[:, idx] if v.ndim == 2 else v[idx]) for k, v in flat.items()})
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
