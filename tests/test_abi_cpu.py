"""Host-side checks of the C-ABI library (no GPU needed): symbols, argument
validation, phase fields, and the symbolic plan driven through a CPU simulation
of the multifrontal LDL^T on the oracle's element matrices."""
import ctypes as C
import json
import os

import numpy as np
import pytest

import oracle
from paper_1908_08292_amd import rve

HERE = os.path.dirname(__file__)


def test_library_exports_every_declared_symbol():
    names = rve.declared_functions()
    assert "rve_solve_batch" in names and "rve_mesh_create" in names and len(names) >= 14
    L = rve.lib()
    for nm in names:
        assert hasattr(L, nm), nm


def test_lame_matches_paper_table():
    tab = json.load(open(os.path.join(HERE, "golden", "lame_table.json")))
    for row in tab["rows"]:
        lam, mu = rve.lame(row["E"], row["nu"])
        assert round(lam, 2) == pytest.approx(row["lambda"], abs=1e-9)
        assert round(mu, 2) == pytest.approx(row["mu"], abs=1e-9)
    with pytest.raises(rve.RveError):
        rve.lame(-1.0, 0.3)


@pytest.mark.parametrize("d,n,r", [(2, 8, 0.25), (2, 16, 0.25), (2, 32, 0.25), (2, 32, 0.1739), (3, 8, 0.3),
                                   (3, 12, 0.2293), (3, 16, 0.4153)])
def test_phase_by_centroid_bit_exact_with_oracle(d, n, r):
    lame_tab = rve.two_phase_lame(10.0)
    m = rve.Mesh(d, n, lame_tab, radius=r)
    assert np.array_equal(m.phase(), oracle.phase_by_centroid(d, n, r))
    m.destroy()


def test_argument_validation():
    lame_tab = rve.two_phase_lame(10.0)
    for bad in [dict(d=4, n=8), dict(d=2, n=1), dict(d=2, n=65), dict(d=3, n=25)]:
        with pytest.raises(rve.RveError) as ei:
            rve.Mesh(bad["d"], bad["n"], lame_tab, radius=0.2)
        assert ei.value.code == rve.RVE_EINVAL
    with pytest.raises(rve.RveError):
        rve.Mesh(2, 4, lame_tab, phase=np.full(16, 5, np.uint8))
    with pytest.raises(rve.RveError):
        rve.Mesh(2, 4, np.array([[1.0, 0.0]]), radius=0.2)   # mu = 0
    m = rve.Mesh(2, 4, lame_tab, radius=0.2)
    h = m.h
    m.destroy()
    assert rve.lib().rve_mesh_destroy(h) == rve.RVE_EINVAL   # double destroy detected
    assert rve.lib().rve_batch_create(None, 4, C.byref(C.c_void_p())) == rve.RVE_EINVAL
    assert rve.lib().rve_solve_batch(None, None, None, None, None, None, None, None, None) == rve.RVE_EINVAL


def test_plan_info_counts():
    info = rve.plan_info(2, 32)
    assert info["nfronts"] > 10 and info["max_front"] <= 2 * 128
    # nested dissection beats the banded (profile) ordering by a wide margin
    assert 5e6 < info["factor_flops"] < 2e7
    assert rve.plan_info(3, 16)["factor_flops"] < 3e10


def simulate_multifrontal(P, d, n, ke, b):
    """numpy replay of the device algorithm on the exported plan."""
    fr = P["fronts"]
    nf = len(fr)
    kmap_end = list(fr[1:, 7]) + [len(P["kpair"])]
    nd = (2 ** d) * d
    stack = {}
    Ls = {}
    for s in range(nf):
        m, p, parent, roff, reloff, cb, ce, kb = fr[s]
        mu = m - p
        rows = P["rows"][roff: roff + m]
        Fp = np.zeros((m, p)); Us = np.zeros((mu, mu)); y = b[rows[:p]].copy(); ru = np.zeros(mu)
        for q in range(kb, kmap_end[s]):
            rn, cn, c0, cc = P["kpair"][q]
            for k in range(d):
                for l in range(d):
                    r, c = rn * d + k, cn * d + l
                    if r < c:
                        continue
                    v = 0.0
                    for e, la, lb in P["kcontrib"][c0: c0 + cc]:
                        v += ke[e][lb * d + k, la * d + l]
                    Fp[r, c] = v
        for ch in P["children"][cb:ce]:
            Uc, ruc = stack.pop(ch)
            mc = Uc.shape[0]
            rel = P["relind"][fr[ch][4]: fr[ch][4] + mc]
            for i in range(mc):
                for k in range(i + 1):
                    R, Cc = rel[i], rel[k]
                    if Cc < p:
                        Fp[R, Cc] += Uc[i, k]
                    else:
                        Us[R - p, Cc - p] += Uc[i, k]
                if rel[i] < p:
                    y[rel[i]] += ruc[i]
                else:
                    ru[rel[i] - p] += ruc[i]
        Dg = np.zeros(p)
        for j in range(p):
            piv = Fp[j, j]
            col = Fp[j + 1:, j].copy()
            for k in range(j + 1, p):
                Fp[k:, k] -= col[k - j - 1:] * col[k - j - 1] / piv
            l = col / piv
            y[j + 1:] -= l[: p - j - 1] * y[j]
            ru -= l[p - j - 1:] * y[j]
            Fp[j + 1:, j] = l
            Dg[j] = piv
        L21 = Fp[p:, :]
        Us -= (L21 * Dg) @ L21.T
        stack[s] = (np.tril(Us) + np.tril(Us, -1).T, ru)
        Ls[s] = (rows, Fp, Dg, y)
    x = np.zeros_like(b)
    for s in range(nf - 1, -1, -1):
        rows, Fp, Dg, y = Ls[s]
        p = Fp.shape[1]
        v = y / Dg - Fp[p:, :].T @ x[rows[p:]]
        xs = np.linalg.solve(np.tril(Fp[:p, :p], -1).T + np.eye(p), v)
        x[rows[:p]] = xs
    return x


@pytest.mark.parametrize("d,n", [(2, 2), (2, 4), (2, 8), (2, 16), (3, 2), (3, 4), (3, 5)])
def test_plan_drives_a_correct_multifrontal_solve(d, n):
    rng = np.random.default_rng(d * 100 + n)
    lame_tab = oracle.two_phase_lame(10.0)
    phase = rng.integers(0, 2, n ** d).astype(np.uint8)
    F = np.eye(d) + rng.uniform(-0.1, 0.1, (d, d))
    w = rng.uniform(-0.02, 0.02, d * n ** d) / n
    ke = [oracle.element(d, n, phase, lame_tab, e, F, w)[2] for e in range(n ** d)]
    st, Rf, K, dw = oracle.debug_system(d, n, phase, lame_tab, F, w)
    b = np.zeros(d * n ** d)
    b[d:] = rng.normal(size=K.shape[0])
    x = simulate_multifrontal(rve.plan_export(d, n), d, n, ke, b)
    ref = np.linalg.solve(K, b[d:])
    assert np.abs(x[d:] - ref).max() < 1e-9 * np.abs(ref).max()
    assert np.all(x[:d] == 0)


@pytest.mark.parametrize("d,n", [(2, 12), (2, 16), (2, 24), (2, 32), (3, 3), (3, 4)])
def test_workgroup_front_schedule(d, n):
    """Every workgroup front is processed once, after its children; the 1, 2 or 4
    fronts sharing a step are independent, have equal pivot and child counts
    (the kernel's thread groups then pass the same barriers), at most 128 rows
    each, and fit the front region (largest packed front plus its rhs rows and
    diagonal) together, also with their staged panels and FP64 scratch in the
    backward substitution."""
    sch = rve.plan_schedule(d, n)
    e = rve.plan_export(d, n)
    fr, ch = e["fronts"], e["children"]
    m, p, cb, ce = fr[:, 0], fr[:, 1], fr[:, 5], fr[:, 6]
    wave = sch["wave"].astype(bool)
    done = wave.copy()
    seen = np.zeros(len(fr), int)
    mm = int(m.max())
    region = mm * (mm + 1) // 2 + mm * (d * d + 1)
    sizes = []
    for step in sch["steps"]:
        fs = [int(s) for s in step if s >= 0]
        assert len(fs) in (1, 2, 4) and list(step[:len(fs)]) == fs
        sizes.append(len(fs))
        for s in fs:
            assert not wave[s]
            assert all(done[ch[q]] for q in range(cb[s], ce[s])), step
            seen[s] += 1
        if len(fs) > 1:
            assert len({(p[s], ce[s] - cb[s]) for s in fs}) == 1
            assert max(m[s] for s in fs) <= 128
            assert sum(m[s] * (m[s] + 1) // 2 + m[s] * (d * d + 1) for s in fs) <= region
            panel = [p[s] * m[s] - p[s] * (p[s] - 1) // 2 for s in fs]
            assert sum(panel) + sum(2 * (d * d * m[s] + 3 * p[s]) + 1 for s in fs) <= region
        done[fs] = True
    assert np.all(seen[~wave] == 1) and np.all(seen[wave] == 0)
    if (d, n) == (2, 32):
        # the 24 small separator fronts: 16 of at most 78 rows four at a time, 8 in pairs
        assert sorted(sizes, reverse=True)[:8] == [4, 4, 4, 4, 2, 2, 2, 2] and len(sizes) == 15


def test_fehmm_symbols_exported():
    from paper_1908_08292_amd import fehmm
    names = fehmm.declared_functions()
    assert "fehmm_macro_step" in names and "fehmm_set_surrogate" in names and len(names) == 11
    L = fehmm.lib()
    for nm in names:
        assert hasattr(L, nm), nm


def test_surrogate_symbols_and_validation():
    from paper_1908_08292_amd import surrogate as S
    names = S.declared_functions()
    assert "rve_surrogate_train" in names and "rve_surrogate_eval" in names and len(names) == 11
    L = S.lib()
    for nm in names:
        assert hasattr(L, nm), nm
    assert "rve_solve_batch_subset" in rve.declared_functions()
    o = S.train_opts()
    assert o.steps == 80000 and o.batch == 3840 and o.precision == S.BF16X3
    assert abs(o.lr - 2e-3) < 1e-9 and abs(o.beta2 - 0.999) < 1e-7
    # argument checks run before any device call
    with pytest.raises(rve.RveError) as e:
        S.Surrogate(np.eye(4), c_scale=(0.5, -1.0, 0.5))
    assert e.value.code == rve.RVE_EINVAL
    with pytest.raises(rve.RveError) as e:
        S.Surrogate(np.eye(4), w_scale=0.0)
    assert e.value.code == rve.RVE_EINVAL
    bad = np.eye(4)
    bad[0, 0] = np.nan
    with pytest.raises(rve.RveError):
        S.Surrogate(bad)
    assert L.rve_surrogate_select(None, 10, 1e-3, None, None, None) == rve.RVE_EINVAL
    assert L.rve_surrogate_eval(None, None, None, None, None, 0, 1, None) == rve.RVE_EINVAL


@pytest.mark.parametrize("d,n,leaf,wave", [(2, 8, 4, 64), (2, 16, 8, 32), (2, 16, 32, 0), (3, 4, 8, 64),
                                            (3, 5, 64, 0)])
def test_tuned_plans_drive_a_correct_multifrontal_solve(d, n, leaf, wave):
    """Every plan the autotuner can choose (other leaf sizes of the dissection,
    other wave-per-front limits) still eliminates the periodic system exactly."""
    rve.tuning_set(d, n, leaf=leaf, wave_max_m=wave, slots=0)
    try:
        assert rve.tuning_get(d, n)["leaf"] == leaf
        rng = np.random.default_rng(d * 1000 + n + leaf)
        lame_tab = oracle.two_phase_lame(10.0)
        phase = rng.integers(0, 2, n ** d).astype(np.uint8)
        F = np.eye(d) + rng.uniform(-0.1, 0.1, (d, d))
        w = rng.uniform(-0.02, 0.02, d * n ** d) / n
        ke = [oracle.element(d, n, phase, lame_tab, e, F, w)[2] for e in range(n ** d)]
        st, Rf, K, dw = oracle.debug_system(d, n, phase, lame_tab, F, w)
        b = np.zeros(d * n ** d)
        b[d:] = rng.normal(size=K.shape[0])
        plan = rve.plan_export(d, n)
        x = simulate_multifrontal(plan, d, n, ke, b)
        ref = np.linalg.solve(K, b[d:])
        assert np.abs(x[d:] - ref).max() < 1e-9 * np.abs(ref).max()
    finally:
        rve.tuning_reset(d, n)
    assert rve.tuning_get(d, n) == dict(leaf=0, wave_max_m=64, slots=0, threads=0, ms=0.0)


def test_tuning_validation():
    with pytest.raises(rve.RveError):
        rve.tuning_set(2, 8, leaf=-1)
    with pytest.raises(rve.RveError):
        rve.tuning_set(2, 8, wave_max_m=65)
    with pytest.raises(rve.RveError):
        rve.tuning_set(2, 8, threads=384)
    rve.tuning_set(2, 8, threads=512)
    try:
        assert rve.tuning_get(2, 8)["threads"] == 512
    finally:
        rve.tuning_reset(2, 8)
    with pytest.raises(rve.RveError):
        rve.tuning_get(4, 8)
    assert "rve_autotune" in rve.declared_functions()
