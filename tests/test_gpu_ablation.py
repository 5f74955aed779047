"""GPU parity (through the C ABI) of the paper's kernel families rebuilt as
ablations: the four k-NN kernels and the four projection kernels.

They work in plain FP32 (the paper's precision), so the bar is FP32's: the
four k-NN kernels evaluate every distance with the same fused multiply-adds
in dimension order and must agree with each other entry for entry; against
the FP64 oracle, neighbour sets must match wherever the oracle's k-th and
(k+1)-th squared distances differ by more than FP32 can resolve (4 (d + 2) u
relative), and distances to FP32 rounding.  The projections from the
oracle's neighbours must lie within 1e-4 of the grid span of the oracle's
output (the 2-D path's bar) on the paper-shaped data, and agree with each
other to 2e-5 of the span there (elsewhere FP32 systems of poorly conditioned
points differ more between summation orders; each is held to the oracle's bar
on all but the worst 0.1% of points)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
ALGOS = ("base", "shared", "gridinsert", "bitonic")
PROJ = ("base", "shared", "aligned", "registers")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _paper_shaped(d, n):
    from paper_2201_00701_amd import synth
    w = synth.paper_shaped(d, n=max(n, 4096))
    return w.X[:n], w.L, w.l, w.k


CASES = [("paper d16", 16, 20000, None, None, None), ("paper d32", 32, 20000, None, None, None),
         ("ragged k5", 7, 1001, 100, 10, 5), ("k20 g300", 24, 3000, 300, 20, 20)]


def _case(label, d, n, g, cols, k):
    from paper_2201_00701_amd import synth
    if g is None:
        return _paper_shaped(d, n)
    X = synth.mixture(n + g, d, 6, seed=d + g)
    L = synth.landmarks_from_data(X, g, seed=g)
    return np.ascontiguousarray(X[:n]), L, synth.grid2d(g, cols), k


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_ablation_knn_parity(torch_dev, oracle_mod, case):
    from paper_2201_00701_amd import esom
    label, d = case[0], case[1]
    X, L, l, k = _case(*case)
    g = len(L)
    res = {}
    for algo in ALGOS:
        _say("case ablation knn %s %s n=%d d=%d g=%d k=%d" % (label, algo, len(X), d, g, k))
        idx, d2 = esom.ablation_knn(algo, _dev(torch_dev, X), _dev(torch_dev, L), k)
        torch_dev.cuda.synchronize()
        res[algo] = (idx.cpu().numpy(), d2.cpu().numpy())
    for algo in ALGOS[1:]:
        np.testing.assert_array_equal(res[algo][0], res["base"][0], err_msg=algo)
        np.testing.assert_array_equal(res[algo][1], res["base"][1], err_msg=algo)
    ridx, rd2 = oracle_mod.knn(X, L, min(k + 1, g), threads=8)
    gi, gd = res["base"]
    if k < g:
        tie = (rd2[:, k] - rd2[:, k - 1]) <= 4 * (d + 2) * U32 * rd2[:, k]
    else:
        tie = np.zeros(len(X), bool)
    same = np.all(np.sort(gi, 1) == np.sort(ridx[:, :k], 1), axis=1)
    _say("  set mismatches %d outside %d FP32 ties" % (int(np.sum(~same & ~tie)), int(tie.sum())))
    assert np.all(same | tie)
    ok = same
    np.testing.assert_allclose(gd[ok], rd2[ok, :k], rtol=4 * (d + 2) * U32, atol=1e-30)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_ablation_projection_parity(torch_dev, oracle_mod, case):
    from paper_2201_00701_amd import esom
    label, d = case[0], case[1]
    X, L, l, k = _case(*case)
    ref = oracle_mod.embed(X, L, l, k, threads=8)
    idx = ref["idx"][:, :k].astype(np.int32)
    d2 = ref["d2"][:, :k].astype(np.float32)
    span = float(np.ptp(l, axis=0).max())
    outs = {}
    for algo in PROJ:
        _say("case ablation projection %s %s n=%d d=%d k=%d" % (label, algo, len(X), d, k))
        o = esom.ablation_project(algo, _dev(torch_dev, X), _dev(torch_dev, L), _dev(torch_dev, l),
                                  _dev(torch_dev, idx), _dev(torch_dev, d2))
        torch_dev.cuda.synchronize()
        outs[algo] = o.cpu().numpy().astype(np.float64)
        err = np.abs(outs[algo] - ref["out"]).max(axis=1)
        _say("  max_err=%.3g mean_err=%.3g tol=%.3g" % (err.max(), err.mean(), 1e-4 * span))
        if label.startswith("paper"):
            assert err.max() <= 1e-4 * span
        else:
            # FP32 systems: the bar on the points the FP64 solution holds to a
            # modest condition, the rest reported
            assert np.quantile(err, 0.999) <= 1e-4 * span
    if label.startswith("paper"):
        # well-conditioned systems: the four orders of FP32 summation agree closely
        for algo in PROJ[1:]:
            assert np.abs(outs[algo] - outs["base"]).max() <= 2e-5 * span, algo


def test_ablation_invalid_arguments(torch_dev):
    from paper_2201_00701_amd import esom
    X = _dev(torch_dev, np.zeros((10, 8), np.float32))
    L = _dev(torch_dev, np.zeros((20, 8), np.float32))
    idx = torch_dev.zeros((10, 4), dtype=torch_dev.int32, device="cuda")
    d2 = torch_dev.zeros((10, 4), dtype=torch_dev.float32, device="cuda")
    assert esom.esom_ablation_knn(7, X.data_ptr(), 10, 8, L.data_ptr(), 20, 4, idx.data_ptr(),
                                  d2.data_ptr()) == esom.ESOM_EINVAL
    assert esom.esom_ablation_knn(0, X.data_ptr(), 10, 8, L.data_ptr(), 20, 21, idx.data_ptr(),
                                  d2.data_ptr()) == esom.ESOM_EINVAL
    assert esom.esom_ablation_knn(0, X.data_ptr(), 10, 300, L.data_ptr(), 20, 4, idx.data_ptr(),
                                  d2.data_ptr()) == esom.ESOM_EINVAL
