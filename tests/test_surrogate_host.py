"""Host logic of the surrogate driver (no GPU): the gate calibration rule,
input features and the grouping of samples by star and spot."""
import numpy as np
import pytest

import workloads as W

S = pytest.importorskip("paper_2301_04259_amd.surrogate", reason="libsoap.so not built")


def _accepted(c, spread, thr):
    return c * np.asarray(spread) < thr


def test_calibration_meets_the_miss_rate_and_accepts_the_most():
    rng = np.random.default_rng(0)
    n, thr = 4000, 1e-4
    spread = 10.0 ** rng.uniform(-7, -3.5, n)
    err = np.abs(rng.normal(0, 1, n)) * spread * 3.0
    for alpha in (0.0, 1e-3, 1e-2):
        c = S.calib_for_miss_rate(err, spread, thr, alpha)
        acc = _accepted(c, spread, thr)
        assert acc.any()
        assert np.sum(err[acc] >= thr) <= alpha * acc.sum()
        # brute force over factors between consecutive sample thresholds:
        # none accepts more within the rate
        ts = np.sort(thr / spread)
        cands = np.concatenate([[0.5 * ts[0]], np.sqrt(ts[:-1] * ts[1:]), [2.0 * ts[-1]]])
        best = 0
        for cc in cands:
            a = _accepted(cc, spread, thr)
            if a.sum() > best and np.sum(err[a] >= thr) <= alpha * a.sum():
                best = a.sum()
        assert acc.sum() == best


def test_calibration_edge_cases():
    thr = 1.0
    # every sample fine: all accepted
    c = S.calib_for_miss_rate([0.1, 0.2, 0.3], [1.0, 2.0, 3.0], thr, 0.0)
    assert _accepted(c, [1.0, 2.0, 3.0], thr).all()
    # the most confident sample is wrong and alpha = 0: nothing accepted
    c = S.calib_for_miss_rate([5.0, 0.1], [0.1, 1.0], thr, 0.0)
    assert not _accepted(c, [0.1, 1.0], thr).any()


def test_features_geometry():
    # a spot at the disk centre of an equator-on star: x = y = 0, z = 1
    f = S.features([0.0], [0.0], [0.055], [0.6], [0.0], [5500.0], [90.0], [3.0])[0]
    assert f.shape == (12,)
    np.testing.assert_allclose(f[[0, 1, 2, 3, 4, 5]], [0, 0, 1, 0, 0, 1], atol=1e-7)
    np.testing.assert_allclose(f[[6, 7, 8, 9, 10, 11]], [0, 0, 0, 1, 0, 1], atol=1e-7)
    # longitude and phase enter only through lon + 360 phase
    a = S.features([20.0], [100.0], [0.05], [0.5], [0.25], [5000.0], [60.0], [2.0])
    b = S.features([20.0], [190.0], [0.05], [0.5], [0.0], [5000.0], [60.0], [2.0])
    np.testing.assert_allclose(a, b, atol=1e-6)
    # pole-on star: the pole sits at the disk centre
    p = S.features([90.0], [37.0], [0.05], [0.5], [0.3], [5000.0], [0.0], [2.0])[0]
    np.testing.assert_allclose(p[[3, 4, 5]], [0.0, 0.0, 1.0], atol=1e-7)


def test_samples_grouped_by_star_and_spot():
    smp = W.cfg5_multi_samples(40, n_per=8, seed=3)
    assert np.all(np.diff(smp.star) >= 0)  # spots ordered by star
    idx = np.sort(np.random.default_rng(1).choice(smp.n, 100, replace=False))
    sid = S.sample_stars(smp, idx)
    assert np.all(np.diff(sid) >= 0)  # any sorted subset stays grouped
    starts, ends = S._groups(sid)
    assert starts[0] == 0 and ends[-1] == len(idx)
    for a, b in zip(starts, ends):
        assert len(set(sid[a:b])) == 1
    t, i, v = smp.star_params(smp.star)
    assert set(np.unique(t)) <= set(W.CFG5_TEFF) and set(np.unique(i)) <= set(W.CFG5_INCL)
    assert set(np.unique(v)) <= set(W.CFG5_VSINI)


def test_star_rows_lookup_matches_the_id_map():
    st = S.Stars()
    rng = np.random.default_rng(3)
    ids = rng.permutation(5000)[:300]
    for i, sid in enumerate(ids):
        st.add(int(sid), None, 5000.0 + i, 60.0, 2.0)
    q = rng.choice(ids, 2000)
    assert np.array_equal(st.rows(q), np.array([st.row[int(v)] for v in q], dtype=np.int32))
    st.add(int(ids[0]), None, 1.0, 1.0, 1.0)  # re-added id: the latest row wins, as in the map
    assert st.rows([ids[0]])[0] == st.row[int(ids[0])] == 300
    missing = int(np.setdiff1d(np.arange(5000), ids)[0])
    with pytest.raises(KeyError):
        st.rows([ids[1], missing])
    assert len(S.Stars().rows([])) == 0


def test_fit_basis_falls_back_when_the_svd_does_not_converge(monkeypatch):
    rng = np.random.default_rng(4)
    D = rng.standard_normal((40, 30)) @ np.diag(np.linspace(3.0, 0.1, 30))
    mean0, V0 = S.fit_basis(D, 5)

    def fail(*a, **k):
        raise np.linalg.LinAlgError("SVD did not converge")

    monkeypatch.setattr(np.linalg, "svd", fail)
    mean1, V1 = S.fit_basis(D, 5)
    assert np.array_equal(mean0, mean1)
    # the same axes up to sign
    assert np.allclose(np.abs(np.sum(V0 * V1, axis=0)), 1.0, atol=1e-10)
    with pytest.raises(ValueError):
        S.fit_basis(np.full((3, 4), np.nan), 2)
