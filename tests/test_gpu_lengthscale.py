"""Length-scale study (Sec. 3.3) as batched dataset generation on the HIP path.

The 16^3 four-sphere cell with the Tab. 3 constants is swept over the
elastic and plastic lengths l_e, l_p in [0.1, 1], every cell one RVE of a
resident batch.  Checks:
  - two cells of the batch (FP64) against the oracle, response curves to 1e-10
    on the same iteration schedule;
  - the paper's description of the heat maps: M11(t_last) is about constant
    over the sweep; T32(t_last) falls as either length grows (stiffer when
    l_e is small, harder to yield when l_p is small); at l_e = l_p = 0.1 the
    response is Cauchy-like with T32 near 14 and M11 near 0.5 (the paper's
    printed values, from its own four-sphere placement, which is not given:
    a loose check, not a parity pin); the corner l_e = 1, l_p = 0.1 does not
    yield at the macro level in the simulation window.
  - the mixed-precision batch of a 10 x 10 sweep: every cell converges, and
    its final T32, M11 stay near the FP64 values.
"""
import time

import numpy as np
import pytest

from oracle import micropolar as O
from paper_2409_10774_amd import workloads as W

pytestmark = pytest.mark.gpu

T32, M11, P = 7, 9, 36
SHAPE = (16, 16, 16)


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_10774_amd import mp as _mp
    return _mp


def say(*a):
    print(*a, flush=True)


def sweep(mp, les, lps, precision):
    cells = [W.length_scale_rve(le, lp) for le in les for lp in lps]
    B = mp.Batch([SHAPE], arena_bytes=2 << 30, precision=precision, max_rves=len(cells))
    ids = [B.admit(w.phase_map, w.phases, w.times, w.E, w.G, tol=w.tol, h=w.h) for w in cells]
    t0 = time.perf_counter()
    launches = B.drain()
    dt = time.perf_counter() - t0
    q = [B.query(i) for i in ids]
    recs = [B.responses(i) for i in ids]
    B.close()
    its = sum(qq[3] for qq in q)
    say(f"{precision} sweep of {len(cells)} cells: {dt:.2f} s, {len(cells) / dt:.1f} RVE solves/s, "
        f"{its * 16 ** 3 / dt:.3e} voxel-iterations/s, {launches} graph launches")
    assert all(qq[1] == mp.MP_OK and qq[2] == len(w.E) for qq, w in zip(q, cells)), q
    return cells, recs


def test_length_scale_sweep_fp64(mp):
    say("case: length-scale sweep, 4 x 4 cells, FP64 batch")
    les = lps = [0.1, 0.4, 0.7, 1.0]
    cells, recs = sweep(mp, les, lps, "fp64")
    last = np.array([r[-1] for r in recs])
    t32 = last[:, T32].reshape(4, 4)          # [le][lp]
    m11 = last[:, M11].reshape(4, 4)
    say("T32(t_last) rows l_e = 0.1 .. 1, columns l_p = 0.1 .. 1\n", np.round(t32, 3))
    say("M11(t_last)\n", np.round(m11, 4))
    # two cells against the oracle
    for k in (0, 12):      # (0.1, 0.1), (1.0, 0.1)
        w, rec = cells[k], recs[k]
        it_gpu = [int(v) for v in rec[:, 41]]
        run = lambda sched: O.Solver(w.phase_map, w.phases, h=w.h, tol=w.tol).solve(
            w.times, w.E, w.G, schedule=sched)
        out = run(None)
        if out["iters"] != it_gpu:
            n = sum(a != b for a, b in zip(out["iters"], it_gpu))
            say(f"{w.name}: {n} step(s) with different iteration counts; oracle on the GPU schedule")
            assert n <= 3
            out = run(it_gpu)
        ref = out["resp"]
        scale = np.abs(ref).max(axis=0)
        big = scale > 1e-12 * scale.max()
        curve = (np.abs(rec[:, :40] - ref)[:, big].max(axis=0) / scale[big]).max()
        say(f"{w.name}: curves vs oracle max rel {curve:.2e}")
        assert curve < 1e-10
    assert (m11.max() - m11.min()) < 0.05 * m11.mean()
    assert np.all(np.diff(t32, axis=1) <= 1e-12)                  # softer as l_p grows
    assert np.all(np.diff(t32[:, :2], axis=0) < 0)                # stiffer for small l_e ...
    assert np.all(t32[0] > t32[-1])                               # ... in every column
    assert 12.0 < t32[0, 0] < 16.0 and 0.45 < m11[0, 0] < 0.55
    assert np.all(recs[12][:, P] == 0.0)


def test_length_scale_sweep_mixed_dataset(mp):
    say("case: length-scale sweep, 10 x 10 cells, mixed-precision batch")
    les = lps = list(np.round(np.linspace(0.1, 1.0, 10), 3))
    cells, recs = sweep(mp, les, lps, "mixed")
    last = np.array([r[-1] for r in recs])
    ref_cells, ref_recs = sweep(mp, les[::3], lps[::3], "fp64")
    ref = {(w.info["le"], w.info["lp"]): r[-1] for w, r in zip(ref_cells, ref_recs)}
    worst = 0.0
    for w, row in zip(cells, last):
        key = (w.info["le"], w.info["lp"])
        if key in ref:
            for c in (T32, M11):
                worst = max(worst, abs(row[c] - ref[key][c]) / abs(ref[key][c]))
    say(f"mixed vs FP64 final T32, M11: max rel {worst:.2e}")
    assert worst < 1e-3
