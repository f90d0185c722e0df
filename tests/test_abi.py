"""Host-side checks of the C ABI (no GPU needed): every entry point declared
in include/mp.h is exported by the built library, and problem validation
(workspace sizing runs no device code) rejects what it must."""
import math
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "mp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mp_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2409_10774_amd import mp
    names = declared()
    assert "mp_plan_create" in names and "mp_solve_load_path" in names
    out = subprocess.run(["nm", "-D", "--defined-only", mp.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\b(mp_[a-z_]+)\b", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(mp.lib, n)


def base_problem(**kw):
    from paper_2409_10774_amd import mp, workloads as W
    wl = W.single_sphere_16()
    phases = kw.pop("phases", wl.phases)
    pm = kw.pop("phase_map", wl.phase_map)
    return mp.make_problem(pm, phases, **kw)


def test_workspace_size_scales_with_grid():
    from paper_2409_10774_amd import mp
    n = mp.mp_plan_workspace_size(base_problem())
    # 18 spectra + 4 x 18 real fields + 4 scalar fields, FP64, 16^3 voxels
    assert n >= (18 + 4 * 18 + 4) * 8 * 16 ** 3


@pytest.mark.parametrize("change,msg", [
    (dict(tol=0.0), "tol"),
    (dict(max_iter=0), "max_iter"),
    (dict(h=-1.0), "h must"),
])
def test_rejects_bad_problem(change, msg):
    from paper_2409_10774_amd import mp
    with pytest.raises(mp.MPError) as ei:
        mp.mp_plan_workspace_size(base_problem(**change))
    assert ei.value.status == mp.MP_E_INVALID and msg in str(ei.value)


def bad_phase(**kw):
    from paper_2409_10774_amd import workloads as W
    p = W.matrix_phase()
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("kw", [dict(kappa=0.0), dict(mu=-1.0), dict(beta=5.0, gamma=4.0),
                                dict(alpha=0.1), dict(tY=0.0), dict(a1=0.0), dict(lam=math.nan),
                                dict(tH=-0.1)])
def test_rejects_bad_phase(kw):
    from paper_2409_10774_amd import mp, workloads as W
    wl = W.single_sphere_16()
    with pytest.raises(mp.MPError) as ei:
        mp.mp_plan_workspace_size(base_problem(phases=[bad_phase(**kw), wl.phases[1]]))
    assert ei.value.status == mp.MP_E_INVALID


@pytest.mark.parametrize("shape", [(16, 16, 10), (16, 14, 16), (5, 16, 16), (16, 16, 512), (2, 4, 4), (16, 16, 20)])
def test_rejects_unsupported_grid(shape):
    from paper_2409_10774_amd import mp, workloads as W
    wl = W.single_sphere_16()
    with pytest.raises(mp.MPError):
        mp.mp_plan_workspace_size(base_problem(phase_map=np.zeros(shape, np.uint8)))


def test_accepts_beta_equal_gamma_and_elastic_alpha():
    from paper_2409_10774_amd import mp
    p = bad_phase(alpha=0.3, tY=math.inf, mY=math.inf)    # alpha allowed when micro-elastic
    assert mp.mp_plan_workspace_size(base_problem(phases=[p, p])) > 0


def test_mixed_workspace_layout():
    """Per voxel, FP64: half spectra 144 B, strain state and its previous
    step 2 x 144, history base 144, committed stresses 144, p, q twice 32, the
    phase id 1 (753 B); mixed: the spectra, base and committed stresses in
    FP32 (3 x 72 less), the strain state still FP64 (537 B)."""
    from paper_2409_10774_amd import mp
    a = mp.mp_plan_workspace_size(base_problem())
    b = mp.mp_plan_workspace_size(base_problem(precision="mixed"))
    n = 16 ** 3
    assert 753 * n <= a < 753 * n + 64 * 1024
    assert 537 * n <= b < 537 * n + 64 * 1024


def test_batch_footprint_and_validation():
    """Batch admission sizing runs on the host: the footprint covers the
    plan layout plus the load path and step records, grows with the step
    count, stores the spectra, base and stresses in FP32 in the mixed form,
    and rejects bad input."""
    from paper_2409_10774_amd import mp, workloads as W
    wl = W.single_sphere_16()
    prob = mp.make_problem(wl.phase_map, wl.phases, precision="fp64")
    cfg64 = mp.batch_config([(16, 16, 16)], precision="fp64")
    cfg32 = mp.batch_config([(16, 16, 16)], precision="mixed")

    def fp(cfg, p, n_steps):
        n = mp.C.c_size_t()
        st = mp.lib.mp_batch_footprint(mp.C.byref(cfg), mp.C.byref(p), n_steps, mp.C.byref(n))
        return st, n.value

    st, f10 = fp(cfg64, prob, 10)
    assert st == mp.MP_OK
    assert f10 >= mp.mp_plan_workspace_size(prob)
    st, f100 = fp(cfg64, prob, 100)
    # 90 more steps: 19 more path doubles and 48 more record doubles each
    assert f100 - f10 >= 90 * (19 + 48) * 8 - 512
    pmix = mp.make_problem(wl.phase_map, wl.phases, precision="mixed")
    st, fmix = fp(cfg32, pmix, 10)
    assert st == mp.MP_OK and f10 - fmix >= 3 * 72 * 16 ** 3
    assert fp(cfg64, prob, 0)[0] == mp.MP_E_INVALID
    bad = mp.make_problem(wl.phase_map, wl.phases, tol=0.0)
    assert fp(cfg64, bad, 10)[0] == mp.MP_E_INVALID


def test_batch_create_rejects_bad_config():
    """Configuration errors are found before any device work."""
    from paper_2409_10774_amd import mp
    h = mp.C.c_void_p()
    for kw, shapes in [(dict(max_rves=0), [(16, 16, 16)]), (dict(max_rves=513), [(16, 16, 16)]),
                       (dict(iters_per_launch=0), [(16, 16, 16)]), ({}, [(16, 16, 17)]),
                       ({}, [(16, 16, 16), (16, 16, 16)]), ({}, [])]:
        cfg = mp.batch_config(shapes, **kw)
        st = mp.lib.mp_batch_create(mp.C.byref(cfg), mp.C.c_void_p(256), 1 << 30, None, mp.C.byref(h))
        assert st == mp.MP_E_INVALID, (kw, shapes, st)


def aniso_problem(**change):
    """16^3 sphere cell whose inclusion carries Eq. 5 tensors."""
    from paper_2409_10774_amd import workloads as W
    wl = W.single_sphere_16()
    inc = W.anisotropic_phase(5, t_scale=3.0, m_scale=4.0)
    for k, v in change.items():
        setattr(inc, k, v)
    return base_problem(phases=[wl.phases[0], inc])


def test_accepts_anisotropic_elastic_phase():
    from paper_2409_10774_amd import mp
    p = aniso_problem()
    assert p.n_aniso == 1 and p.aniso[0].phase == 1
    assert mp.mp_plan_workspace_size(p) >= mp.mp_plan_workspace_size(base_problem())


def _asym(A):
    A = np.array(A, copy=True)
    A[0, 1, 2, 2] += 0.5          # breaks A_klmn = A_mnkl
    return A


@pytest.mark.parametrize("change,msg", [
    (dict(tY=1.0), "must be elastic"),
    (dict(mY=1.0), "must be elastic"),
    ("asym", "symmetric positive definite"),
    ("indef", "symmetric positive definite"),
])
def test_rejects_bad_anisotropic_phase(change, msg):
    from paper_2409_10774_amd import mp, workloads as W
    if change == "asym":
        change = dict(A=_asym(W.anisotropic_phase(5).A))
    elif change == "indef":
        B = -np.eye(9).reshape(3, 3, 3, 3)
        change = dict(B=B)
    with pytest.raises(mp.MPError) as ei:
        mp.mp_plan_workspace_size(aniso_problem(**change))
    assert ei.value.status == mp.MP_E_INVALID and msg in str(ei.value)


def test_batch_footprint_of_anisotropic_phase():
    """A batch takes Eq. 5 phases (the footprint grows by their row
    matrices) and tensor reference media (and by the symbol)."""
    from paper_2409_10774_amd import mp
    cfg = mp.batch_config([(16, 16, 16)], precision="fp64")
    n = mp.C.c_size_t()
    st = mp.lib.mp_batch_footprint(mp.C.byref(cfg), mp.C.byref(base_problem()), 3, mp.C.byref(n))
    plain = n.value
    p = aniso_problem()
    st = mp.lib.mp_batch_footprint(mp.C.byref(cfg), mp.C.byref(p), 3, mp.C.byref(n))
    assert st == mp.MP_OK and n.value >= plain
    aniso = n.value
    p.ref_mode = mp.MP_REF_TENSOR_PHASE_MEAN
    st = mp.lib.mp_batch_footprint(mp.C.byref(cfg), mp.C.byref(p), 3, mp.C.byref(n))
    assert st == mp.MP_OK and n.value >= aniso


def test_tensor_mean_reference_validation():
    """MP_REF_TENSOR_MEAN, MP_REF_TENSOR_PHASE_MEAN: accepted with Eq. 5 and
    Eq. 6 phases, also with beta = gamma (the workspace gains the reference's
    row matrices and symbol coefficients); an unknown mode is rejected."""
    from paper_2409_10774_amd import mp, workloads as W
    plain = mp.mp_plan_workspace_size(aniso_problem())
    p = aniso_problem()
    p.ref_mode = mp.MP_REF_TENSOR_MEAN
    assert mp.mp_plan_workspace_size(p) >= plain
    # beta = gamma in every phase of the sphere cell: <B> has no skew
    # stiffness, the symbol stays positive definite through <A>
    assert all(ph.beta == ph.gamma for ph in W.single_sphere_16().phases)
    iso = base_problem(ref_mode="tensor_mean")
    assert mp.mp_plan_workspace_size(iso) > 0
    p.ref_mode = mp.MP_REF_TENSOR_PHASE_MEAN
    assert mp.mp_plan_workspace_size(p) >= plain
    p.ref_mode = 6
    with pytest.raises(mp.MPError) as ei:
        mp.mp_plan_workspace_size(p)
    assert ei.value.status == mp.MP_E_INVALID and "ref_mode" in str(ei.value)


def test_augmented_lagrangian_validation():
    """The augmented-Lagrangian scheme's problems are checked on the host:
    FP64 only, 0 < relax < 2, an isotropic reference, and a penalty with
    gamma0 > beta0 unless every phase present has gamma = beta."""
    from paper_2409_10774_amd import mp, workloads as W
    ok = base_problem(scheme="al", ref_mode="geometric_mean", relax=1.7)
    assert mp.mp_plan_workspace_size(ok) > 0           # beta = gamma everywhere
    for kw, msg in [(dict(precision="mixed"), "FP64"), (dict(relax=2.0), "relax"),
                    (dict(relax=0.0), "relax"), (dict(ref_mode="tensor_mean"), "isotropic")]:
        args = dict(scheme="al", ref_mode="geometric_mean", relax=1.7)
        args.update(kw)
        with pytest.raises(mp.MPError) as ei:
            mp.mp_plan_workspace_size(base_problem(**args))
        assert ei.value.status == mp.MP_E_INVALID and msg in str(ei.value), (kw, str(ei.value))
    skew = W.matrix_phase()
    skew.beta = 0.5 * skew.gamma
    wl = W.single_sphere_16()
    with pytest.raises(mp.MPError) as ei:
        mp.mp_plan_workspace_size(base_problem(phases=[skew, wl.phases[1]], scheme="al", ref_mode="explicit",
                                               ref=(1.0, 1.0, 0.1, 0.0, 2.0, 2.0)))
    assert ei.value.status == mp.MP_E_INVALID and "gamma0 > beta0" in str(ei.value)
    assert mp.mp_plan_workspace_size(base_problem(phases=[skew, wl.phases[1]], scheme="al",
                                                  ref_mode="geometric_mean")) > 0


def test_stored_green_workspace_and_validation():
    """MP_GREEN_STORED adds the inverse-symbol table to a plan's workspace
    and to a batched RVE's footprint: 21 words of the bulk precision per
    frequency of the half spectrum (n0/2 n1 n2), plus the reference's symbol
    coefficients; other green_mode values are rejected."""
    from paper_2409_10774_amd import mp, workloads as W
    nspec = 8 * 16 * 16
    for prec, w in (("fp64", 8), ("mixed", 4)):
        a = mp.mp_plan_workspace_size(base_problem(precision=prec))
        b = mp.mp_plan_workspace_size(base_problem(precision=prec, green="stored"))
        assert 21 * nspec * w <= b - a < 21 * nspec * w + 4096, (prec, b - a)
    p = base_problem()
    p.green_mode = 2
    with pytest.raises(mp.MPError) as ei:
        mp.mp_plan_workspace_size(p)
    assert ei.value.status == mp.MP_E_INVALID and "green_mode" in str(ei.value)
    cfg = mp.batch_config([(16, 16, 16)], precision="fp64")
    fp = []
    for green in ("computed", "stored"):
        n = mp.C.c_size_t()
        st = mp.lib.mp_batch_footprint(mp.C.byref(cfg), mp.C.byref(base_problem(green=green)), 4, mp.C.byref(n))
        assert st == mp.MP_OK
        fp.append(n.value)
    assert 21 * nspec * 8 <= fp[1] - fp[0] < 21 * nspec * 8 + 4096
