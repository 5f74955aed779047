"""Pins for the FP64 oracle against facts that do not come from the oracle itself.

* k-NN: brute force with scipy's distance routine and a lexicographic sort.
* scores: the hand-computed vector in tests/golden/tscore.txt, plus the
  properties the paper states (highest for the closest, zero at the k-th
  when k < g) and scale invariance.
* projection: exact recovery for similarity-embedded landmarks (every
  residual of the paper's objective vanishes), an independent least-squares
  solve of the stacked weighted residuals, invariances, continuity.
* landmark update: scikit-learn's Lloyd step, scipy's vector quantiser, and a
  per-point weighted mean for the batch SOM.
"""
import os

import numpy as np
import pytest
from scipy.spatial.distance import cdist

HERE = os.path.dirname(os.path.abspath(__file__))


def _dyadic(a, q=64):
    """Round to multiples of 1/q so float32 holds the values exactly."""
    return (np.round(np.asarray(a, np.float64) * q) / q).astype(np.float32)


def _random_problem(rng, n=40, d=5, g=12, dyadic=False):
    X = rng.normal(size=(n, d)) * 2
    L = rng.normal(size=(g, d)) * 2
    l = rng.uniform(-3, 3, size=(g, 2))
    if dyadic:
        return _dyadic(X), _dyadic(L), _dyadic(l)
    return X.astype(np.float32), L.astype(np.float32), l.astype(np.float32)


# ---------------------------------------------------------------- k-NN step


@pytest.mark.parametrize("seed", range(6))
def test_knn_matches_bruteforce(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    n, d, g = 150, 3, 17
    # integer coordinates make exact distance ties common
    X = rng.integers(-3, 4, size=(n, d)).astype(np.float32)
    L = rng.integers(-3, 4, size=(g, d)).astype(np.float32)
    L[5] = L[2]  # duplicate landmark
    m = 9
    idx, d2 = oracle_mod.knn(X, L, m)
    D2 = cdist(X.astype(np.float64), L.astype(np.float64), "sqeuclidean")
    for i in range(n):
        order = np.lexsort((np.arange(g), D2[i]))[:m]
        assert list(idx[i]) == list(order)
        np.testing.assert_array_equal(d2[i], D2[i][order])


def test_knn_strided_rows(oracle_mod):
    rng = np.random.default_rng(3)
    Xbig = rng.normal(size=(30, 9)).astype(np.float32)
    X = Xbig[:, :6]  # row stride 9 floats
    L = rng.normal(size=(8, 6)).astype(np.float32)
    a, da = oracle_mod.knn(X, L, 4)
    b, db = oracle_mod.knn(np.ascontiguousarray(X), L, 4)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(da, db)


# ---------------------------------------------------------------- scores


def test_scores_hand_computed(oracle_mod):
    rows = [l for l in open(os.path.join(HERE, "golden", "tscore.txt")) if not l.startswith("#")]
    vals = [float(v) for v in rows[0].split()]
    delta, expect = vals[:3], vals[3:]
    s, deg = oracle_mod.scores(delta, g=10, boost=1.0, cutoff=10.0)
    assert not deg
    np.testing.assert_allclose(s, expect, rtol=2e-6, atol=1e-12)
    assert s[2] == 0.0


@pytest.mark.parametrize("k,g", [(3, 10), (8, 64), (16, 400), (20, 1024), (5, 5)])
def test_score_properties(oracle_mod, k, g):
    rng = np.random.default_rng(k * 7 + g)
    for _ in range(20):
        delta = np.sort(rng.uniform(0.1, 10.0, k))
        s, deg = oracle_mod.scores(delta, g)
        assert not deg
        assert np.all(np.diff(s) <= 0), "closest landmark must score highest"
        if k < g:
            assert s[-1] == 0.0, "k-th landmark must score exactly 0 when k < g"
            assert np.all(s[:-1] > 0)
        else:
            assert np.all(s > 0), "no cutoff when k == g"
        s2, _ = oracle_mod.scores(delta * 3.7, g)
        np.testing.assert_allclose(s2, s, rtol=1e-12, atol=1e-300)


def test_score_boost_flattens(oracle_mod):
    delta = np.array([1.0, 1.5, 2.0, 2.2, 3.0])
    s1, _ = oracle_mod.scores(delta, 5, boost=1.0)
    s0, _ = oracle_mod.scores(delta, 5, boost=0.1)
    assert (s0[0] / s0[-1]) < (s1[0] / s1[-1])


def test_scores_all_equal_is_degenerate(oracle_mod):
    s, deg = oracle_mod.scores([2.0, 2.0, 2.0, 2.0], 10)
    assert deg and np.all(s == 0)


def _golden_e():
    # e-factors of the hand-computed case delta = (1, 2, 3) (tests/golden/tscore.txt)
    return np.array([2.281785, 0.624125, 0.170714])


@pytest.mark.parametrize("t,flat", [(1e-9, False), (2.0 ** -52, True), (2.0 ** -51, True)])
def test_scores_flat_spread(oracle_mod, t, flat):
    # delta = 1 + t (0, 1, 2) is a positive affine image of the golden (1, 2, 3):
    # the standardised exponent (mu - delta_i) / sigma is invariant under such
    # maps, so the e-factors equal the golden ones while the variance is
    # resolvable (t = 1e-9: sigma^2 ~ 6e-19 mu^2).  Below the flat-variance
    # threshold (sigma^2 <= 1e-30 mu^2, spreads of a few units in the last place
    # of double) every e-factor is 1: the scores are the cutoff factors alone.
    delta = np.array([1.0, 1.0 + t, 1.0 + 2.0 * t])
    s, deg = oracle_mod.scores(delta, g=10, boost=1.0, cutoff=10.0)
    assert not deg
    c = 1.0 - np.exp(10.0 * (delta / delta[2] - 1.0))
    assert c[0] > 0 and c[1] > 0 and s[2] == 0.0
    e = s[:2] / c[:2]
    if flat:
        np.testing.assert_allclose(e, [1.0, 1.0], rtol=1e-12)
    else:
        np.testing.assert_allclose(e, _golden_e()[:2], rtol=2e-5)


# ---------------------------------------------------------------- projection


def _similarity_problem(rng, g=20, d=6, exact=True):
    """L_j = c Q l_j + t with Q orthonormal (d x 2).  With ``exact`` every value
    is a small dyadic rational so float32 stores it exactly."""
    l = rng.integers(-4, 5, size=(g, 2)).astype(np.float64)
    l += rng.integers(0, 4, size=(g, 2)) / 4.0
    if exact:
        perm = rng.permutation(d)
        Q = np.zeros((d, 2))
        Q[perm[0], 0] = rng.choice([-1, 1])
        Q[perm[1], 1] = rng.choice([-1, 1])
        c = 2.0
        t = rng.integers(-5, 6, size=d).astype(np.float64)
    else:
        Q, _ = np.linalg.qr(rng.normal(size=(d, 2)))
        c = 1.7
        t = rng.normal(size=d)
    L = c * l @ Q.T + t
    return L, l, Q, c, t


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("k", [3, 5, 8])
def test_exact_recovery_similarity(oracle_mod, seed, k):
    rng = np.random.default_rng(seed)
    L, l, Q, c, t = _similarity_problem(rng)
    n, d = 25, L.shape[1]
    P = rng.integers(-12, 13, size=(n, 2)) / 4.0
    noise = rng.integers(-3, 4, size=(n, d)) / 2.0
    noise -= (noise @ Q) @ Q.T  # orthogonal to the landmark plane (exact here)
    X = c * P @ Q.T + t + noise
    L32, l32, X32 = L.astype(np.float32), l.astype(np.float32), X.astype(np.float32)
    assert np.array_equal(X32.astype(np.float64), X) and np.array_equal(L32.astype(np.float64), L)
    for boost, adjust in [(1.0, 1.0), (0.5, 0.0), (2.0, 2.0)]:
        r = oracle_mod.embed(X32, L32, l32, k, boost=boost, adjust=adjust, gravity=0.0)
        ok = np.ones(n, bool)
        if k == 3:
            # one active pair: p is only determined along that pair's line
            ok[:] = False
        err = np.abs(r["out"] - P).max(axis=1)
        assert np.all(err[ok] < 1e-10), err.max()
        # with gravity the answer moves by O(eps): the shift scales linearly
        e6 = np.abs(oracle_mod.embed(X32, L32, l32, k, boost=boost, adjust=adjust,
                                     gravity=1e-6)["out"] - P).max(axis=1)
        e8 = np.abs(oracle_mod.embed(X32, L32, l32, k, boost=boost, adjust=adjust,
                                     gravity=1e-8)["out"] - P).max(axis=1)
        big = ok & (e8 > 1e-9) & (e6 < 1e-3)  # linear regime
        np.testing.assert_allclose(e8[big] * 100, e6[big], rtol=0.05)


def test_point_on_landmark_maps_to_its_2d_position(oracle_mod):
    rng = np.random.default_rng(11)
    L, l, Q, c, t = _similarity_problem(rng, g=30)
    X = L.copy()
    r = oracle_mod.embed(X.astype(np.float32), L.astype(np.float32), l.astype(np.float32), 6,
                         gravity=0.0)
    np.testing.assert_allclose(r["out"], l, atol=1e-10)


def test_recovery_general_rotation(oracle_mod):
    rng = np.random.default_rng(21)
    L, l, Q, c, t = _similarity_problem(rng, g=25, d=9, exact=False)
    P = rng.uniform(-3, 3, size=(30, 2))
    X = c * P @ Q.T + t
    r = oracle_mod.embed(X.astype(np.float32), L.astype(np.float32), l.astype(np.float32), 7,
                         gravity=0.0)
    # float32 rounding of the inputs is the only error source
    np.testing.assert_allclose(r["out"], P, atol=2e-4)


def _lstsq_reference(X, L, l, k, idx, s, adjust, gravity, drop_kth=False):
    """Solve argmin_p sum w (D - d(p))^2 + gravity terms with numpy.linalg.lstsq on
    the stacked weighted rows (independent of the oracle's normal equations)."""
    X = X.astype(np.float64); L = L.astype(np.float64); l = l.astype(np.float64)
    out = np.zeros((len(X), 2))
    for i in range(len(X)):
        A, b = [], []
        kk = k - 1 if drop_kth else k
        for a_ in range(kk):
            for b_ in range(a_ + 1, kk):
                u, v = idx[i, a_], idx[i, b_]
                H = L[v] - L[u]
                HH = H @ H
                h = l[v] - l[u]
                hh = h @ h
                if HH == 0 or hh == 0:
                    continue
                D = (X[i] - L[u]) @ H / HH
                w = s[i, a_] * s[i, b_] * hh ** (1.0 - adjust)
                sw = np.sqrt(w)
                A.append(sw * h / hh)
                b.append(sw * (D + h @ l[u] / hh))
        for a_ in range(k):
            sg = np.sqrt(gravity * s[i, a_])
            A.append([sg, 0.0]); b.append(sg * l[idx[i, a_], 0])
            A.append([0.0, sg]); b.append(sg * l[idx[i, a_], 1])
        out[i] = np.linalg.lstsq(np.array(A), np.array(b), rcond=None)[0]
    return out


@pytest.mark.parametrize("k,g,adjust", [(3, 12, 1.0), (4, 12, 1.0), (6, 12, 0.5), (12, 12, 1.0),
                                        (7, 30, 1.3)])
def test_normal_equations_match_lstsq(oracle_mod, k, g, adjust):
    rng = np.random.default_rng(k * 100 + g)
    X, L, l = _random_problem(rng, n=30, d=5, g=g)
    L[3] = L[1]  # duplicate HD landmark: its pair must be skipped
    l[7] = l[4]  # duplicate 2-D landmark
    r = oracle_mod.embed(X, L, l, k, adjust=adjust, gravity=1e-3)
    idx = r["idx"][:, :k]
    s = np.stack([oracle_mod.scores(np.sqrt(r["d2"][i, :k]), g)[0] for i in range(len(X))])
    ref = _lstsq_reference(X, L, l, k, idx, s, adjust, 1e-3)
    np.testing.assert_allclose(r["out"], ref, rtol=1e-9, atol=1e-9)
    if k < g:
        # pairs with the k-th neighbour carry zero weight
        ref2 = _lstsq_reference(X, L, l, k, idx, s, adjust, 1e-3, drop_kth=True)
        np.testing.assert_allclose(r["out"], ref2, rtol=1e-9, atol=1e-9)


def test_invariances_exact(oracle_mod):
    rng = np.random.default_rng(5)
    X, L, l = _random_problem(rng, n=60, d=6, g=25, dyadic=True)
    k = 7
    base = oracle_mod.embed(X, L, l, k)["out"]
    # (i) common translation of X and L (integer shift: exact in float32)
    t = rng.integers(-4, 5, size=6).astype(np.float32)
    np.testing.assert_allclose(oracle_mod.embed(X + t, L + t, l, k)["out"], base, atol=1e-9)
    # (ii) orthogonal transform: signed coordinate permutation (exact)
    perm, sign = rng.permutation(6), rng.choice([-1, 1], 6).astype(np.float32)
    np.testing.assert_allclose(oracle_mod.embed(X[:, perm] * sign, L[:, perm] * sign, l, k)["out"],
                               base, atol=1e-9)
    # (iii) uniform scaling of X and L
    np.testing.assert_allclose(oracle_mod.embed(X * 4, L * 4, l, k)["out"], base, atol=1e-9)
    # (iv) translating l shifts the output
    tau = np.array([3.0, -2.0], np.float32)
    np.testing.assert_allclose(oracle_mod.embed(X, L, l + tau, k)["out"], base + tau, atol=1e-9)
    # (v) rotating / reflecting l by a quarter turn and a mirror
    R = np.array([[0, -1], [1, 0]], np.float32)
    np.testing.assert_allclose(oracle_mod.embed(X, L, l @ R.T, k)["out"], base @ R.T, atol=1e-9)
    Mr = np.array([[1, 0], [0, -1]], np.float32)
    np.testing.assert_allclose(oracle_mod.embed(X, L, l @ Mr.T, k)["out"], base @ Mr.T, atol=1e-9)
    # (vi) scaling l scales the output (without the gravity term)
    b0 = oracle_mod.embed(X, L, l, k, gravity=0.0)["out"]
    np.testing.assert_allclose(oracle_mod.embed(X, L, l * 2, k, gravity=0.0)["out"], b0 * 2,
                               atol=1e-9)
    # (vii) landmark order (L and l permuted together)
    pg = rng.permutation(25)
    r = oracle_mod.embed(X, L, l, k)
    gap = r["d2"][:, k] - r["d2"][:, k - 1]
    ok = gap > 1e-9
    rp = oracle_mod.embed(X, L[pg], l[pg], k)["out"]
    np.testing.assert_allclose(rp[ok], base[ok], atol=1e-9)


def test_invariances_general_rotation(oracle_mod):
    rng = np.random.default_rng(8)
    X, L, l = _random_problem(rng, n=40, d=7, g=30)
    k = 8
    base = oracle_mod.embed(X, L, l, k)["out"]
    Q, _ = np.linalg.qr(rng.normal(size=(7, 7)))
    t = rng.normal(size=7) * 10
    Xr = (X.astype(np.float64) @ Q.T + t).astype(np.float32)
    Lr = (L.astype(np.float64) @ Q.T + t).astype(np.float32)
    np.testing.assert_allclose(oracle_mod.embed(Xr, Lr, l, k)["out"], base, atol=2e-3)


def test_continuity_along_a_path(oracle_mod):
    """The k-th neighbour scores exactly zero, so the output must not jump when a
    neighbour enters or leaves the k-neighbourhood: zooming in on each change
    of the neighbour set, the output change shrinks with the step."""
    from paper_2201_00701_amd import synth
    X = synth.mixture(400, 5, 4, seed=3, sd_range=(0.5, 1.5), background=0.0)
    L = synth.landmarks_from_data(X, 36, seed=3)
    l = synth.grid2d(36, 6)
    k = 6
    x0, x1 = X[0].astype(np.float64), X[1].astype(np.float64)
    ts = np.linspace(0, 1, 2001)
    path = ((1 - ts)[:, None] * x0 + ts[:, None] * x1).astype(np.float32)
    r = oracle_mod.embed(path, L, l, k)
    change = np.nonzero(np.any(np.sort(r["idx"][1:, :k], 1) != np.sort(r["idx"][:-1, :k], 1),
                               axis=1))[0]
    assert len(change) >= 3  # the neighbourhood really changes along the path
    for i in change:
        lo, hi = ts[i], ts[i + 1]
        fine = np.linspace(lo, hi, 257)
        pf = ((1 - fine)[:, None] * x0 + fine[:, None] * x1).astype(np.float32)
        out = oracle_mod.embed(pf, L, l, k)["out"]
        jumps = np.linalg.norm(np.diff(out, axis=0), axis=1)
        coarse = np.linalg.norm(r["out"][i + 1] - r["out"][i])
        # a discontinuity would keep a jump of the full coarse size at one fine step
        assert jumps.max() < 0.1 * coarse + 1e-6, (i, jumps.max(), coarse)


def test_all_equidistant_maps_to_centroid(oracle_mod):
    X = np.zeros((1, 3), np.float32)
    L = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [5, 5, 5], [6, 6, 6]],
                 np.float32)
    l = np.array([[0, 0], [2, 0], [0, 4], [2, 4], [9, 9], [8, 8]], np.float32)
    r = oracle_mod.embed(X, L, l, 4)
    np.testing.assert_allclose(r["out"][0], [1.0, 2.0])
    assert r["n_degenerate"] == 1


def test_rank_deficient_system_maps_to_centroid(oracle_mod):
    """k = 3 leaves one weighted pair: without gravity the 2x2 system has rank
    one and det = 0 up to rounding (of either sign), so every point maps to the
    centroid of its neighbours' 2-D positions.  Collinear 2-D neighbours do the
    same at larger k.  With gravity the same points are solved."""
    rng = np.random.default_rng(5)
    X, L, l = _random_problem(rng, n=60, d=5, g=30)
    r = oracle_mod.embed(X, L, l, 3, gravity=0.0)
    cent = l[r["idx"][:, :3]].astype(np.float64).mean(1)
    np.testing.assert_allclose(r["out"], cent, rtol=0, atol=1e-12)
    assert r["n_degenerate"] == len(X)
    r1 = oracle_mod.embed(X, L, l, 3)
    assert r1["n_degenerate"] == 0
    assert np.all(np.abs(r1["out"] - cent).max(1) > 1e-3)
    # all landmarks on one line in 2-D: every pair direction is the same
    l_line = np.stack([np.arange(30, dtype=np.float32), np.zeros(30, np.float32)], 1)
    r2 = oracle_mod.embed(X, L, l_line, 6, gravity=0.0)
    np.testing.assert_allclose(r2["out"], l_line[r2["idx"][:, :6]].astype(np.float64).mean(1),
                               rtol=0, atol=1e-12)


def test_invalid_arguments(oracle_mod):
    X = np.zeros((2, 3), np.float32)
    L = np.zeros((5, 3), np.float32)
    l = np.zeros((5, 2), np.float32)
    with pytest.raises(ValueError):
        oracle_mod.embed(X, L, l, 2)
    with pytest.raises(ValueError):
        oracle_mod.embed(X, L, l, 6)


# ---------------------------------------------------------------- landmark update


def _blob_data(seed, n=3000, d=4, g=9):
    rng = np.random.default_rng(seed)
    centers = rng.uniform(-10, 10, size=(g, d))
    X = (centers[rng.integers(0, g, n)] + rng.normal(size=(n, d))).astype(np.float32)
    L = (centers + rng.normal(scale=0.5, size=(g, d))).astype(np.float32)
    l = np.stack([np.arange(g) % 3, np.arange(g) // 3], 1).astype(np.float32)
    return X, L, l


def test_kmeans_alpha1_is_one_lloyd_step(oracle_mod):
    from sklearn.cluster import KMeans
    from scipy.cluster.vq import vq
    X, L, l = _blob_data(1)
    Lnew, counts = oracle_mod.landmark_update(X, L, l, "kmeans", alpha=1.0)
    codes, _ = vq(X.astype(np.float64), L.astype(np.float64))
    assert np.array_equal(np.bincount(codes, minlength=len(L)), counts)
    assert counts.min() > 0
    km = KMeans(n_clusters=len(L), init=L.astype(np.float64), n_init=1, max_iter=1,
                algorithm="lloyd", tol=0.0).fit(X.astype(np.float64))
    np.testing.assert_allclose(Lnew, km.cluster_centers_, rtol=1e-9, atol=1e-9)
    assert counts.sum() == len(X)


def test_kmeans_alpha_blend_and_empty_landmark(oracle_mod):
    X, L, l = _blob_data(2)
    L = np.concatenate([L, np.full((1, L.shape[1]), 1e4, np.float32)])  # owns no point
    l = np.concatenate([l, [[5, 5]]]).astype(np.float32)
    L1, c1 = oracle_mod.landmark_update(X, L, l, "kmeans", alpha=1.0)
    La, ca = oracle_mod.landmark_update(X, L, l, "kmeans", alpha=0.1)
    assert c1[-1] == 0
    np.testing.assert_allclose(La[-1], L[-1])
    np.testing.assert_allclose(La[:-1], L[:-1] + 0.1 * (L1[:-1] - L[:-1]), rtol=1e-12, atol=1e-9)


def test_som_small_sigma_equals_kmeans(oracle_mod):
    X, L, l = _blob_data(3)
    a, _ = oracle_mod.landmark_update(X, L, l, "kmeans", alpha=0.3)
    b, _ = oracle_mod.landmark_update(X, L, l, "som", alpha=0.3, sigma=1e-3)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12)


def test_som_sigma_zero_is_lloyd_step(oracle_mod):
    # sigma = 0: each landmark's neighbourhood is itself alone, so the SOM step
    # is the alpha-blended Lloyd step; a landmark that owns no point stays put
    from scipy.cluster.vq import vq
    X, L, l = _blob_data(6)
    L = np.concatenate([L, np.full((1, L.shape[1]), 1e4, np.float32)])
    l = np.concatenate([l, [[5, 5]]]).astype(np.float32)
    alpha = 0.3
    Lnew, counts = oracle_mod.landmark_update(X, L, l, "som", alpha=alpha, sigma=0.0)
    codes, _ = vq(X.astype(np.float64), L.astype(np.float64))
    assert np.array_equal(np.bincount(codes, minlength=len(L)), counts)
    assert counts[-1] == 0
    L64 = L.astype(np.float64)
    expect = L64.copy()
    for j in range(len(L) - 1):
        mean = X[codes == j].astype(np.float64).mean(0)
        expect[j] = L64[j] + alpha * (mean - L64[j])
    np.testing.assert_allclose(Lnew, expect, rtol=1e-12, atol=1e-12)


def test_som_is_neighbourhood_weighted_mean(oracle_mod):
    from scipy.cluster.vq import vq
    X, L, l = _blob_data(4)
    sigma = 1.1
    Lnew, _ = oracle_mod.landmark_update(X, L, l, "som", alpha=1.0, sigma=sigma)
    codes, _ = vq(X.astype(np.float64), L.astype(np.float64))
    l64 = l.astype(np.float64)
    for j in range(len(L)):
        h = np.exp(-((l64[j] - l64[codes]) ** 2).sum(1) / (2 * sigma * sigma))
        np.testing.assert_allclose(Lnew[j], np.average(X.astype(np.float64), axis=0, weights=h),
                                   rtol=1e-9, atol=1e-9)


def test_landmark_update_point_order_invariant(oracle_mod):
    X, L, l = _blob_data(5)
    perm = np.random.default_rng(0).permutation(len(X))
    a, ca = oracle_mod.landmark_update(X, L, l, "som", alpha=0.5, sigma=0.8)
    b, cb = oracle_mod.landmark_update(X[perm], L, l, "som", alpha=0.5, sigma=0.8)
    assert np.array_equal(ca, cb)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12)


def test_threads_do_not_change_results(oracle_mod):
    rng = np.random.default_rng(9)
    X, L, l = _random_problem(rng, n=500, d=6, g=40)
    a = oracle_mod.embed(X, L, l, 9, threads=1)
    b = oracle_mod.embed(X, L, l, 9, threads=4)
    np.testing.assert_array_equal(a["out"], b["out"])
    np.testing.assert_array_equal(a["idx"], b["idx"])


# ---------------------------------------------------------------- FP32 distances and the cutoff

def _project_given_scores(x, L, l, nb, s, adjust, gravity=1e-5):
    """Normal equations of the pair objective for given scores (FP64)."""
    M = np.zeros((2, 2))
    r = np.zeros(2)
    x = x.astype(np.float64)
    for i in range(len(nb)):
        for j in range(i + 1, len(nb)):
            Lu, Lv = L[nb[i]].astype(np.float64), L[nb[j]].astype(np.float64)
            H = Lv - Lu
            D = (x - Lu) @ H / (H @ H)
            lu = l[nb[i]].astype(np.float64)
            h = l[nb[j]].astype(np.float64) - lu
            hh = h @ h
            q = s[i] * s[j] * hh ** -adjust
            M += q * np.outer(h, h) / hh
            r += q * h * (D + h @ lu / hh)
    for i in range(len(nb)):
        M += gravity * s[i] * np.eye(2)
        r += gravity * s[i] * l[nb[i]]
    return np.linalg.solve(M, r)


def _fp32_d2(x, row):
    acc = np.float32(0)
    for a, b in zip(x, row):
        e = np.float32(a - b)
        acc = np.float32(acc + np.float32(e * e))
    return float(acc)


@pytest.mark.parametrize("k,rows,expect_over", [(3, range(0, 512, 2), True), (16, range(0, 256, 8), False)])
def test_cutoff_weight_sensitivity_to_fp32_distances(oracle_mod, k, rows, expect_over):
    """Scores from FP32-rounded distances, everything else in FP64.  With one
    weighted pair (k = 3, adjust = 0) and the (k-1)-th distance within 1e-8 to
    1e-3 of the k-th, some outputs move past 1e-4 of the grid span (the GPU
    path recomputes such weights from FP64 distances); with k = 16 the other
    pairs hold both directions and the same rounding stays far below it."""
    import sys
    sys.path.insert(0, HERE)
    from test_gpu_parity import _near_cutoff_problem
    oracle = oracle_mod
    X, L, l = _near_cutoff_problem() if k == 3 else _near_cutoff_problem(n=256, m=k, seed=29 + k)
    span = float(max(np.ptp(l[:, 0]), np.ptp(l[:, 1])))
    ref = oracle.embed(X, L, l, k, adjust=0.0, threads=4)
    errs = []
    for p in rows:
        nb = ref["idx"][p][:k]
        s64, _ = oracle.scores(np.sqrt(ref["d2"][p][:k]), len(L))
        d2f = np.array([_fp32_d2(X[p], L[j]) for j in nb])
        s32, _ = oracle.scores(np.sqrt(d2f), len(L))
        errs.append(np.abs(_project_given_scores(X[p], L, l, nb, s32, 0.0)
                           - _project_given_scores(X[p], L, l, nb, s64, 0.0)).max())
    worst = max(errs) / (1e-4 * span)
    if expect_over:
        assert worst > 1.0
    else:
        assert worst < 0.01


# ---------------------------------------------------------------- online SOM training


def _som_problem(seed, n=2000, d=5, side=6):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, d)).astype(np.float32) * 2
    g = side * side
    L = rng.normal(size=(g, d)).astype(np.float32)
    j = np.arange(g)
    l = np.stack([j % side, j // side], 1).astype(np.float32)
    return rng, X, L, l


def _kohonen_serial(X, L, l, rows, sigma, alpha):
    """Textbook online SOM: one point per step, every landmark moves towards it by
    alpha h(j, b) (x - L_j); the landmarks are kept in float32 between steps."""
    L = L.astype(np.float32).copy()
    l64 = l.astype(np.float64)
    for t, r in enumerate(rows):
        x = X[r].astype(np.float64)
        L64 = L.astype(np.float64)
        b = int(np.argmin(((x - L64) ** 2).sum(1)))
        r2 = ((l64 - l64[b]) ** 2).sum(1)
        h = (r2 == 0).astype(np.float64) if sigma[t] == 0 else np.exp(-r2 / (2 * sigma[t] ** 2))
        L = (L64 + alpha[t] * h[:, None] * (x - L64)).astype(np.float32)
    return L


def test_som_train_batch_of_one_is_serial_online_rule(oracle_mod):
    rng, X, L, l = _som_problem(31)
    T = 60
    rows = rng.integers(0, len(X), T)
    sigma = 2.0 * (0.2 / 2.0) ** (np.arange(T) / (T - 1))      # 2 -> 0.2
    alpha = 0.5 * (0.05 / 0.5) ** (np.arange(T) / (T - 1))     # 0.5 -> 0.05
    sigma[17] = 0.0
    got = oracle_mod.som_train(X, L, l, rows.reshape(T, 1), sigma, alpha)
    expect = _kohonen_serial(X, L, l, rows, sigma, alpha)
    np.testing.assert_allclose(got, expect, rtol=1e-6, atol=1e-6)
    assert np.abs(got - L).max() > 0.1  # the landmarks moved


def test_som_train_batch_step_is_average_of_single_point_updates(oracle_mod):
    rng, X, L, l = _som_problem(32)
    B = 64
    rows = rng.integers(0, len(X), B)
    rows[5] = -1            # presents no point, still counts in the batch size
    rows[9] = len(X) + 3
    sigma, alpha = np.array([1.3]), np.array([0.4])
    got = oracle_mod.som_train(X, L, l, rows.reshape(1, B), sigma, alpha)
    L64 = L.astype(np.float64)
    l64 = l.astype(np.float64)
    moves = np.zeros_like(L64)
    for r in rows:
        if r < 0 or r >= len(X):
            continue
        x = X[r].astype(np.float64)
        b = int(np.argmin(((x - L64) ** 2).sum(1)))
        h = np.exp(-((l64 - l64[b]) ** 2).sum(1) / (2 * 1.3 ** 2))
        moves += 0.4 * h[:, None] * (x - L64)
    np.testing.assert_allclose(got, (L64 + moves / B).astype(np.float32), rtol=1e-6, atol=1e-6)


def test_som_train_frozen_and_zero_rate(oracle_mod):
    rng, X, L, l = _som_problem(33)
    T, B = 5, 50
    rows = rng.integers(0, len(X), (T, B))
    frozen = np.zeros(len(L), np.uint8)
    frozen[[0, 7, 20]] = 1
    got = oracle_mod.som_train(X, L, l, rows, np.full(T, 1.0), np.full(T, 0.3), frozen=frozen)
    np.testing.assert_array_equal(got[[0, 7, 20]], L[[0, 7, 20]])
    assert np.abs(got[1] - L[1]).max() > 0
    same = oracle_mod.som_train(X, L, l, rows, np.full(T, 1.0), np.zeros(T))
    np.testing.assert_array_equal(same, L)


# ---------------------------------------------------------------- new-landmark fit


def _fit_problem(seed, g=40, d=7):
    rng = np.random.default_rng(seed)
    l = rng.uniform(0, 8, (g, 2)).astype(np.float32)
    return rng, l


def test_fit_reproduces_affine_embedding(oracle_mod):
    # landmarks on an affine image of the 2-D plane: the fit is exact there
    rng, l = _fit_problem(41)
    A = rng.normal(size=(7, 2))
    c = rng.normal(size=7)
    L = (l.astype(np.float64) @ A.T + c).astype(np.float32)
    p = rng.uniform(1, 7, (25, 2)).astype(np.float32)
    for kfit, sigma in ((3, 1.0), (8, 0.7), (40, 5.0)):
        got = oracle_mod.fit_landmarks(L, l, p, kfit=kfit, sigma=sigma)
        np.testing.assert_allclose(got, p.astype(np.float64) @ A.T + c, rtol=1e-4, atol=1e-4)


def test_fit_matches_weighted_least_squares(oracle_mod):
    rng, l = _fit_problem(42)
    L = rng.normal(size=(len(l), 7)).astype(np.float32)
    p = rng.uniform(0, 8, (20, 2)).astype(np.float32)
    kfit, sigma = 9, 1.5
    got = oracle_mod.fit_landmarks(L, l, p, kfit=kfit, sigma=sigma)
    l64, L64 = l.astype(np.float64), L.astype(np.float64)
    for q, pq in enumerate(p.astype(np.float64)):
        d2 = ((l64 - pq) ** 2).sum(1)
        nb = np.lexsort((np.arange(len(l)), d2))[:kfit]
        w = np.exp(-d2[nb] / (2 * sigma ** 2))
        Z = np.concatenate([l64[nb], np.ones((kfit, 1))], 1)
        coef, *_ = np.linalg.lstsq(Z * np.sqrt(w)[:, None], L64[nb] * np.sqrt(w)[:, None], rcond=None)
        np.testing.assert_allclose(got[q], np.append(pq, 1.0) @ coef, rtol=1e-9, atol=1e-9)


def test_fit_interpolates_three_neighbours_and_collinear_falls_back(oracle_mod):
    rng, l = _fit_problem(43)
    L = rng.normal(size=(len(l), 7)).astype(np.float32)
    # a new landmark placed on an existing one, fitted from three neighbours
    # (non-collinear): the affine map through three points passes through them
    got = oracle_mod.fit_landmarks(L, l, l[[4, 11]], kfit=3, sigma=1.0)
    np.testing.assert_allclose(got, L[[4, 11]], rtol=1e-9, atol=1e-9)
    # collinear 2-D neighbours determine no affine map: weighted mean
    lc = np.stack([np.arange(6.0), np.zeros(6)], 1).astype(np.float32)
    Lc = rng.normal(size=(6, 7)).astype(np.float32)
    p = np.array([[2.3, 0.7]], np.float32)
    got = oracle_mod.fit_landmarks(Lc, lc, p, kfit=6, sigma=2.0)
    w = np.exp(-((lc.astype(np.float64) - p[0]) ** 2).sum(1) / 8.0)
    np.testing.assert_allclose(got[0], np.average(Lc.astype(np.float64), axis=0, weights=w),
                               rtol=1e-9, atol=1e-9)
    # far from every landmark with a small sigma: still finite (no weight underflows)
    far = oracle_mod.fit_landmarks(L, l, np.array([[500.0, -300.0]], np.float32), kfit=5, sigma=0.1)
    assert np.all(np.isfinite(far))


# ---------------------------------------------------------------- 3-D output

def _similarity_problem3(rng, g=24, d=7):
    """L_j = c Q l_j + t with Q a d x 3 matrix of signed unit columns on distinct
    axes and dyadic 3-D positions, so float32 stores every value exactly."""
    l = rng.integers(-4, 5, size=(g, 3)).astype(np.float64) + rng.integers(0, 4, size=(g, 3)) / 4.0
    perm = rng.permutation(d)
    Q = np.zeros((d, 3))
    for a in range(3):
        Q[perm[a], a] = rng.choice([-1, 1])
    c = 2.0
    t = rng.integers(-5, 6, size=d).astype(np.float64)
    return c * l @ Q.T + t, l, Q, c, t


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("k", [4, 6, 9])
def test_embed3_exact_recovery_similarity(oracle_mod, seed, k):
    # every segment coordinate of x = c Q p* + t + noise (noise orthogonal to Q)
    # equals its 3-D counterpart at p*, so the objective is zero at p*
    rng = np.random.default_rng(300 + seed)
    L, l, Q, c, t = _similarity_problem3(rng)
    n, d = 25, L.shape[1]
    P = rng.integers(-12, 13, size=(n, 3)) / 4.0
    noise = rng.integers(-3, 4, size=(n, d)) / 2.0
    noise -= (noise @ Q) @ Q.T
    X = c * P @ Q.T + t + noise
    X32, L32, l32 = X.astype(np.float32), L.astype(np.float32), l.astype(np.float32)
    assert np.array_equal(X32.astype(np.float64), X)
    r = oracle_mod.embed3(X32, L32, l32, k, gravity=0.0)
    err = np.abs(r["out"] - P).max(axis=1)
    # k = 4 leaves three active neighbours: a plane's worth of pairs, which may
    # not fix all three coordinates; larger k must recover p* exactly
    if k > 4:
        assert np.all(err < 1e-10), err.max()
    # points on landmarks map to their 3-D positions
    r2 = oracle_mod.embed3(L32, L32, l32, 7, gravity=0.0)
    np.testing.assert_allclose(r2["out"], l, atol=1e-10)


def test_embed3_planar_positions_reduce_to_2d(oracle_mod):
    # with every 3-D position in the plane z = 0 the third coordinate decouples
    # (no pair has a z component, gravity pulls z to 0) and x, y solve the 2-D system
    rng = np.random.default_rng(17)
    X, L, l = _random_problem(rng, n=80, d=6, g=30)
    l3 = np.concatenate([l, np.zeros((len(l), 1), np.float32)], axis=1)
    for k in (4, 8, 30):
        r2 = oracle_mod.embed(X, L, l, k)
        r3 = oracle_mod.embed3(X, L, l3, k)
        assert r2["n_degenerate"] == 0 and r3["n_degenerate"] == 0
        np.testing.assert_allclose(r3["out"][:, :2], r2["out"], rtol=1e-11, atol=1e-11)
        assert np.all(r3["out"][:, 2] == 0.0)


def _lstsq_reference3(X, L, l3, k, idx, s, adjust, gravity):
    X = X.astype(np.float64); L = L.astype(np.float64); l3 = l3.astype(np.float64)
    out = np.zeros((len(X), 3))
    for i in range(len(X)):
        A, b = [], []
        for a_ in range(k):
            for b_ in range(a_ + 1, k):
                u, v = idx[i, a_], idx[i, b_]
                H = L[v] - L[u]
                h = l3[v] - l3[u]
                if H @ H == 0 or h @ h == 0:
                    continue
                D = (X[i] - L[u]) @ H / (H @ H)
                sw = np.sqrt(s[i, a_] * s[i, b_] * (h @ h) ** (1.0 - adjust))
                A.append(sw * h / (h @ h))
                b.append(sw * (D + h @ l3[u] / (h @ h)))
        for a_ in range(k):
            sg = np.sqrt(gravity * s[i, a_])
            for c in range(3):
                row = np.zeros(3)
                row[c] = sg
                A.append(row)
                b.append(sg * l3[idx[i, a_], c])
        out[i] = np.linalg.lstsq(np.array(A), np.array(b), rcond=None)[0]
    return out


@pytest.mark.parametrize("k,g,adjust", [(5, 16, 1.0), (8, 16, 0.5), (16, 16, 1.0), (7, 30, 1.4)])
def test_embed3_normal_equations_match_lstsq(oracle_mod, k, g, adjust):
    rng = np.random.default_rng(k * 31 + g)
    X, L, l = _random_problem(rng, n=25, d=5, g=g)
    l3 = np.concatenate([l, rng.normal(size=(g, 1)).astype(np.float32)], axis=1)
    L[3] = L[1]   # duplicate HD landmark: its pair is skipped
    l3[7] = l3[4]  # duplicate 3-D landmark
    r = oracle_mod.embed3(X, L, l3, k, adjust=adjust, gravity=1e-3)
    idx = r["idx"][:, :k]
    s = np.stack([oracle_mod.scores(np.sqrt(r["d2"][i, :k]), g)[0] for i in range(len(X))])
    ref = _lstsq_reference3(X, L, l3, k, idx, s, adjust, 1e-3)
    np.testing.assert_allclose(r["out"], ref, rtol=1e-9, atol=1e-9)


def test_embed3_rotation_and_translation_of_positions(oracle_mod):
    # rotating / translating the 3-D positions rotates / translates the output
    rng = np.random.default_rng(23)
    X, L, l = _random_problem(rng, n=40, d=5, g=20)
    l3 = np.concatenate([l, rng.normal(size=(20, 1)).astype(np.float32)], axis=1).astype(np.float64)
    R, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    tau = np.array([0.5, -1.25, 2.0])
    base = oracle_mod.embed3(X, L, l3.astype(np.float32), 7, gravity=0.0)["out"]
    lr = (l3.astype(np.float32).astype(np.float64) @ R.T + tau).astype(np.float32)
    moved = oracle_mod.embed3(X, L, lr, 7, gravity=0.0)["out"]
    # float32 rounding of the rotated positions is the only difference
    np.testing.assert_allclose(moved, base @ R.T + tau, atol=2e-4)


# ---------------------------------------------------------------- graph-mode supervision

@pytest.mark.parametrize("seed", range(3))
def test_landmark_graph_matches_bruteforce(oracle_mod, seed):
    rng = np.random.default_rng(400 + seed)
    g, d, kg = 40, 3, 6
    L = rng.integers(-3, 4, size=(g, d)).astype(np.float32)  # integer grid: exact ties
    L[5] = L[9]  # an exact duplicate: distance 0 to each other
    nbr, d2 = oracle_mod.landmark_graph(L, kg)
    D = cdist(L.astype(np.float64), L.astype(np.float64), "sqeuclidean")
    for u in range(g):
        others = [v for v in range(g) if v != u]
        order = sorted(others, key=lambda v: (D[u, v], v))[:kg]
        assert list(nbr[u]) == order
        np.testing.assert_array_equal(d2[u], D[u, order])
    assert 9 in nbr[5] and 5 in nbr[9]


def test_landmark_graph_more_slots_than_others(oracle_mod):
    L = np.array([[0, 0], [1, 0], [0, 2]], np.float32)
    nbr, d2 = oracle_mod.landmark_graph(L, 4)
    assert list(nbr[0]) == [1, 2, -1, -1] and np.isinf(d2[0, 2:]).all()


def test_layout_single_spring_reaches_rest_length(oracle_mod):
    # two nodes on one edge, no repulsion: each moves step * (r - rest) toward
    # the other, so with step 1/2 the new distance is exactly the rest length
    L = np.array([[0, 0, 0], [3, 4, 0]], np.float32)         # |L_0 - L_1| = 5
    l = np.array([[0, 0], [8, 0]], np.float32)               # r = 8
    nbr = np.array([[1], [0]], np.int32)                     # the edge in both lists: once
    out = oracle_mod.layout(L, nbr, l, steps=1, scale=0.4, repulsion=0.0, step=0.5, max_move=100)
    # rest length 0.4 * 5 = 2: both move 3 toward each other
    np.testing.assert_allclose(out, [[3, 0], [5, 0]], atol=1e-6)
    # the edge in one list only acts the same way
    out1 = oracle_mod.layout(L, np.array([[1], [-1]], np.int32), l, steps=1, scale=0.4,
                             repulsion=0.0, step=0.5, max_move=100)
    np.testing.assert_array_equal(out1, out)
    # a spring at its rest length exerts nothing
    rest = oracle_mod.layout(L, nbr, np.array([[0, 0], [2, 0]], np.float32), scale=0.4,
                             repulsion=0.0, step=0.5)
    np.testing.assert_array_equal(rest, [[0, 0], [2, 0]])


def test_layout_repulsion_of_two_nodes(oracle_mod):
    L = np.zeros((2, 2), np.float32)
    l = np.array([[0, 0], [1.5, 0]], np.float32)
    nbr = np.array([[-1], [-1]], np.int32)  # no edges
    out = oracle_mod.layout(L, nbr, l, repulsion=0.8, soft=0.5, step=0.25, max_move=100)
    push = 0.25 * 0.8 * 1.5 / (1.5 ** 2 + 0.25)
    np.testing.assert_allclose(out, [[-push, 0], [1.5 + push, 0]], rtol=1e-6)
    # the move is shortened to max_move
    out2 = oracle_mod.layout(L, nbr, l, repulsion=0.8, soft=0.5, step=0.25, max_move=0.01)
    np.testing.assert_allclose(out2, [[-0.01, 0], [1.51, 0]], rtol=1e-6)


def test_layout_invariants(oracle_mod):
    rng = np.random.default_rng(41)
    g, d = 30, 5
    L = rng.normal(size=(g, d)).astype(np.float32)
    l = (rng.normal(size=(g, 2)) * 3).astype(np.float32)
    nbr, _ = oracle_mod.landmark_graph(L, 4)
    kw = dict(scale=0.7, repulsion=0.3, soft=0.2, step=0.05, max_move=1e9)
    out = oracle_mod.layout(L, nbr, l, **kw).astype(np.float64)
    # internal forces cancel in pairs: the centroid stays (no clamp, nothing fixed)
    np.testing.assert_allclose(out.mean(axis=0), l.astype(np.float64).mean(axis=0), atol=1e-5)
    # translation equivariance (integer shift: exact)
    sh = np.array([3, -2], np.float32)
    np.testing.assert_allclose(oracle_mod.layout(L, nbr, l + sh, **kw), out + sh, atol=1e-5)
    # rotation equivariance (a quarter turn is exact)
    rot = np.array([[0, -1], [1, 0]], np.float32)
    np.testing.assert_allclose(oracle_mod.layout(L, nbr, l @ rot.T, **kw), out @ rot.T, atol=1e-5)
    # fixed nodes keep their positions, the others still move
    fixed = np.zeros(g, np.uint8)
    fixed[[2, 7]] = 1
    fo = oracle_mod.layout(L, nbr, l, fixed=fixed, **kw)
    np.testing.assert_array_equal(fo[[2, 7]], l[[2, 7]])
    assert np.all(np.abs(fo[0] - l[0]) > 0)
