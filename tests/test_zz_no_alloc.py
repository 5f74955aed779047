"""The allocation-free embed (esom_embed_noalloc) against the context embed
(esom_embed), both through the C ABI: the same kernels on the same inputs, so
outputs and neighbour lists must agree bit for bit; the shared device scratch
keeps the previous call's contents, so calls run in a row with shrinking
inputs.  The medium case is also held to the oracle's bar (neighbour sets
outside near ties, coordinates within 1e-4 of the grid span)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

REL_TIE = 1e-6
COORD_TOL = 1e-4


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _case(seed, n, d, g, cols, k):
    from paper_2201_00701_amd import synth
    X = synth.mixture(n, d, 30, seed=seed)
    L = synth.landmarks_from_data(X, g, seed=seed)
    l = synth.grid2d(g, cols)
    return X, L, l


def _both(torch, X, L, l, k, mode):
    """(noalloc out, idx, d2), (context out, idx, d2) on the same device inputs."""
    from paper_2201_00701_amd import esom
    Xd = torch.from_numpy(X).cuda()
    Ld = torch.from_numpy(L).cuda()
    ld = torch.from_numpy(l).cuda()
    n, d = X.shape
    g = L.shape[0]
    p = esom.esom_default_params(k=k, mode=mode)
    res = []
    for which in ("noalloc", "context"):
        out = torch.full((n, 2), float("nan"), dtype=torch.float32, device="cuda")
        idx = torch.full((n, k), -7, dtype=torch.int32, device="cuda")
        d2 = torch.full((n, k), float("nan"), dtype=torch.float32, device="cuda")
        stream = torch.cuda.current_stream().cuda_stream
        if which == "noalloc":
            rc = esom.esom_embed_noalloc(Xd.data_ptr(), n, d, d, Ld.data_ptr(), ld.data_ptr(), g, p,
                                         out.data_ptr(), idx.data_ptr(), d2.data_ptr(), stream)
            assert rc == esom.ESOM_OK, esom.esom_last_error()
        else:
            h = esom.esom_create(0, 0)
            try:
                rc = esom.esom_embed(h, Xd.data_ptr(), n, d, d, Ld.data_ptr(), ld.data_ptr(), g, p,
                                     out.data_ptr(), idx.data_ptr(), d2.data_ptr(), stream)
                assert rc == esom.ESOM_OK, esom.esom_last_error()
                torch.cuda.synchronize()
            finally:
                esom.esom_destroy(h)
        torch.cuda.synchronize()
        res.append((out.cpu().numpy(), idx.cpu().numpy(), d2.cpu().numpy()))
    return res


def _same(a, b, label):
    (o1, i1, e1), (o2, i2, e2) = a, b
    assert np.array_equal(i1, i2), "%s: neighbour lists differ at %d points" % (
        label, int(np.sum(np.any(i1 != i2, axis=1))))
    assert np.array_equal(e1.view(np.uint32), e2.view(np.uint32)), "%s: distances differ" % label
    assert np.array_equal(o1.view(np.uint32), o2.view(np.uint32)), "%s: outputs differ at %d points" % (
        label, int(np.sum(np.any(o1.view(np.uint32) != o2.view(np.uint32), axis=1))))


def test_noalloc_equals_context_embed_in_a_row(torch_dev):
    import oracle
    oracle.build(force=False)
    # 1) more points than one chunk of the fixed scratch holds (several chunks),
    #    the largest landmark set the variant takes
    X, L, l = _case(81, 3_500_000, 16, 1024, 32, 8)
    _say("noalloc case 1: n=%d d=16 g=1024 k=8 bf16 (several chunks)" % len(X))
    a, b = _both(torch_dev, X, L, l, 8, "bf16")
    _same(a, b, "case 1")
    del X
    # 2) smaller: the 1M x 32-D shape's landmark set on 200k points, FP32 mode,
    #    also against the oracle
    X, L, l = _case(82, 200_000, 32, 400, 20, 16)
    _say("noalloc case 2: n=%d d=32 g=400 k=16 fp32" % len(X))
    a, b = _both(torch_dev, X, L, l, 16, "fp32")
    _same(a, b, "case 2")
    ref = oracle.embed(X, L, l, 16, threads=8)
    od2 = ref["d2"]
    dk, dk1 = np.sqrt(od2[:, 15]), np.sqrt(od2[:, 16])
    tie = (dk1 - dk) < REL_TIE * dk1
    same = np.all(np.sort(a[1], 1) == np.sort(ref["idx"][:, :16], 1), axis=1)
    assert int(np.sum(~same & ~tie)) == 0
    err = np.abs(a[0].astype(np.float64) - ref["out"]).max()
    _say("  oracle max coordinate error %.3g (tolerance %.3g)" % (err, COORD_TOL * 19))
    assert err <= COORD_TOL * 19
    # 3) smaller again, another shape (ragged n, odd d, k above 16, BF16)
    X, L, l = _case(83, 777, 45, 300, 20, 20)
    _say("noalloc case 3: n=%d d=45 g=300 k=20 bf16" % len(X))
    a, b = _both(torch_dev, X, L, l, 20, "bf16")
    _same(a, b, "case 3")


def test_noalloc_rejects_shapes_beyond_its_limits(torch_dev):
    from paper_2201_00701_amd import esom
    X, L, l = _case(84, 1200, 8, 1100, 40, 8)
    Xd, Ld, ld = (torch_dev.from_numpy(a).cuda() for a in (X, L, l))
    out = torch_dev.empty((100, 2), dtype=torch_dev.float32, device="cuda")
    p = esom.esom_default_params(k=8)
    rc = esom.esom_embed_noalloc(Xd.data_ptr(), 100, 8, 8, Ld.data_ptr(), ld.data_ptr(), 1100, p,
                                 out.data_ptr())
    assert rc == esom.ESOM_EINVAL and "allocation-free" in esom.esom_last_error()
    # n == 0 is a no-op
    rc = esom.esom_embed_noalloc(Xd.data_ptr(), 0, 8, 8, Ld.data_ptr(), ld.data_ptr(), 64, p,
                                 out.data_ptr())
    assert rc == esom.ESOM_OK
