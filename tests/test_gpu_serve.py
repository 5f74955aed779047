"""Serving runtime on the GPU: continuous batching, admission by footprint,
k-nearest cache for 2-D-only edits, captured-frame replay.  Each request's
result must be the same alone and in the mix (the kernels are deterministic
and per point, so bitwise), equal to a direct esom_embed call, and within
the parity bar of the oracle."""
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch


def _req(seed, n, d, g, cols):
    from paper_2201_00701_amd import synth
    X = synth.mixture(n + g, d, 8, seed=seed)
    L = synth.landmarks_from_data(X, g, seed=seed)
    return np.ascontiguousarray(X[:n]), L, synth.grid2d(g, cols)


MIX = [(101, 20000, 16, 100, 10, 8, "bf16"), (102, 3000, 32, 400, 20, 16, "fp32"),
       (103, 50000, 48, 1024, 32, 20, "bf16"), (104, 1234, 32, 100, 10, 16, "fp32"),
       (105, 70000, 16, 400, 20, 8, "bf16"), (106, 999, 48, 400, 20, 20, "fp32")]


def _direct(torch, X, L, l, k, mode):
    from paper_2201_00701_amd.esom import Context
    ctx = Context(0)
    out = ctx.embed(torch.from_numpy(X).cuda(), torch.from_numpy(L).cuda(),
                    torch.from_numpy(l).cuda(), k=k, mode=mode)
    torch.cuda.synchronize()
    r = out.cpu().numpy()
    ctx.close()
    return r


def test_alone_equals_mix_equals_direct(torch_dev, oracle_mod):
    from paper_2201_00701_amd.esom import Server
    reqs = [_req(s, n, d, g, c) + (k, m) for (s, n, d, g, c, k, m) in MIX]
    srv = Server(0, 0, 4)
    _say("case serve alone")
    alone = []
    for X, L, l, k, m in reqs:
        rid = srv.submit(L, l, k=k, mode=m, X=X)
        alone.append(srv.wait(rid, 60000)["out"].copy())
    _say("case serve mix (all submitted at once)")
    rids = [srv.submit(L, l, k=k, mode=m, X=X) for X, L, l, k, m in reqs]
    infos = [srv.wait(r, 60000) for r in rids]
    st = srv.stats()
    _say("  serve stats %s" % st)
    for (X, L, l, k, m), a, inf in zip(reqs, alone, infos):
        np.testing.assert_array_equal(inf["out"], a)
    # overlapping execution: some request started before another finished
    starts = sorted((i["start_ms"], i["done_ms"]) for i in infos)
    assert any(starts[j + 1][0] < starts[j][1] for j in range(len(starts) - 1))
    # equal to a direct esom_embed call, and within the oracle bar
    for idx in (1, 3):
        X, L, l, k, m = reqs[idx]
        np.testing.assert_array_equal(_direct(torch_dev, X, L, l, k, m), alone[idx])
        ref = oracle_mod.embed(X, L, l, k, threads=8)
        span = float(max(np.ptp(l[:, 0]), np.ptp(l[:, 1])))
        assert np.abs(alone[idx] - ref["out"]).max() <= 1e-4 * span
    srv.close()


@pytest.mark.parametrize("k", [16, 8])
def test_resident_dataset_2d_edits_use_cache_and_graph(torch_dev, k):
    # k = 8 also takes the FP64 cutoff-weight refinement, on both paths
    from paper_2201_00701_amd.esom import Server
    rng = np.random.default_rng(7)
    X, L, l0 = _req(201, 40000, 32, 400, 20)
    srv = Server(0, 0, 2)
    did = srv.put(X)
    out = np.empty((len(X), 2), np.float32)
    _say("case serve resident dataset frames k=%d" % k)
    hits, replays = 0, 0
    l = l0.copy()
    for frame in range(8):
        if frame:
            moved = rng.choice(len(l), rng.integers(1, 6), replace=False)
            l = l.copy()
            l[moved] += rng.normal(0, 0.5, (len(moved), 2)).astype(np.float32)
        rid = srv.submit(L, l, k=k, mode="bf16", dataset=did, out=out)
        info = srv.wait(rid, 60000)
        hits += info["cache_hit"]
        replays += info["graph_replay"]
        ref = _direct(torch_dev, X, L, l, k, "bf16")
        np.testing.assert_array_equal(out, ref)
        _say("  frame %d cache_hit=%d graph_replay=%d" % (frame, info["cache_hit"],
                                                           info["graph_replay"]))
    assert hits >= 6 and replays >= 4
    # a high-dimensional change invalidates the cache
    L2 = L.copy()
    L2[0] += 0.25
    rid = srv.submit(L2, l, k=k, mode="bf16", dataset=did, out=out)
    info = srv.wait(rid, 60000)
    assert info["cache_hit"] == 0
    np.testing.assert_array_equal(out, _direct(torch_dev, X, L2, l, k, "bf16"))
    srv.drop(did)
    srv.close()


def test_alternating_datasets_keep_replaying(torch_dev):
    # edits of two resident datasets interleave on a 2-slot server: each slot
    # keeps the graphs of several frames and requests go to the slot that
    # holds their dataset's graph, so both datasets' frames replay
    from paper_2201_00701_amd.esom import Server
    rng = np.random.default_rng(11)
    cases = [_req(211, 30000, 32, 400, 20), _req(212, 20000, 16, 100, 10)]
    srv = Server(0, 0, 2)
    dids = [srv.put(X) for X, _, _ in cases]
    ls = [l.copy() for _, _, l in cases]
    outs = [np.empty((len(X), 2), np.float32) for X, _, _ in cases]
    _say("case serve alternating resident datasets")
    replays = [0, 0]
    for frame in range(14):
        i = frame % 2
        X, L, _ = cases[i]
        if frame >= 2:
            moved = rng.choice(len(ls[i]), 2, replace=False)
            ls[i] = ls[i].copy()
            ls[i][moved] += rng.normal(0, 0.5, (2, 2)).astype(np.float32)
        info = srv.wait(srv.submit(L, ls[i], k=8, mode="bf16", dataset=dids[i], out=outs[i]), 60000)
        replays[i] += info["graph_replay"]
        np.testing.assert_array_equal(outs[i], _direct(torch_dev, X, L, ls[i], 8, "bf16"))
    _say("  replays per dataset %s" % replays)
    assert min(replays) >= 3
    srv.close()


def test_admission_by_footprint(torch_dev):
    from paper_2201_00701_amd import esom
    from paper_2201_00701_amd.esom import Server
    X, L, l = _req(301, 200000, 32, 400, 20)
    # a budget that fits one such request at a time
    budget = 45 << 20
    srv = Server(0, budget, 4)
    _say("case serve admission")
    rids = [srv.submit(L, l, k=16, mode="bf16", X=X) for _ in range(3)]
    infos = [srv.wait(r, 60000) for r in rids]
    st = srv.stats()
    _say("  stats %s" % st)
    assert st["peak_bytes"] <= budget
    for i in infos[1:]:
        np.testing.assert_array_equal(i["out"], infos[0]["out"])
    # serialised by the budget: each started after the previous finished
    iv = sorted((i["start_ms"], i["done_ms"]) for i in infos)
    assert all(iv[j + 1][0] >= iv[j][1] - 1e-3 for j in range(len(iv) - 1))
    # a request that can never fit is refused at submission
    big = np.zeros((4_000_000, 32), np.float32)
    with pytest.raises(esom.EsomError) as e:
        srv.submit(L, l, k=16, X=big)
    assert e.value.code == esom.ESOM_ENOMEM
    srv.close()


def test_drop_while_in_flight_and_unknown_ids(torch_dev):
    from paper_2201_00701_amd import esom
    from paper_2201_00701_amd.esom import Server
    X, L, l = _req(401, 100000, 16, 100, 10)
    srv = Server(0, 0, 2)
    did = srv.put(X)
    out = np.empty((len(X), 2), np.float32)
    _say("case serve drop in flight")
    rid = srv.submit(L, l, k=8, dataset=did, out=out)
    srv.drop(did)
    info = srv.wait(rid, 60000)
    assert info["status"] == 0
    np.testing.assert_array_equal(out, _direct(torch_dev, X, L, l, 8, "fp32"))
    with pytest.raises(esom.EsomError):
        srv.submit(L, l, k=8, dataset=did, out=out)
    rc, _ = esom.esom_serve_wait(srv.handle, 987654321, 0)
    assert rc == esom.ESOM_ENOTFOUND
    srv.close()


def test_resident_nan_row_cache_hit(torch_dev):
    # a non-finite row gets index -1 in the k-nearest cache; the next 2-D edit
    # projects from the cache: that row must go to the exact path again (NaN
    # output, no out-of-range loads) and every other row must equal a direct call
    from paper_2201_00701_amd.esom import Server
    X, L, l = _req(311, 5000, 16, 100, 10)
    X = X.copy()
    X[17, 3] = np.nan
    srv = Server(0, 0, 2)
    did = srv.put(X)
    _say("case serve resident dataset with a NaN row")
    out1 = np.empty((len(X), 2), np.float32)
    info1 = srv.wait(srv.submit(L, l, k=8, mode="bf16", dataset=did, out=out1), 60000)
    l2 = l.copy()
    l2[5] += 0.3
    out2 = np.empty((len(X), 2), np.float32)
    info2 = srv.wait(srv.submit(L, l2, k=8, mode="bf16", dataset=did, out=out2), 60000)
    assert info1["cache_hit"] == 0 and info2["cache_hit"] == 1
    ok = np.arange(len(X)) != 17
    np.testing.assert_array_equal(out1[ok], _direct(torch_dev, X, L, l, 8, "bf16")[ok])
    np.testing.assert_array_equal(out2[ok], _direct(torch_dev, X, L, l2, 8, "bf16")[ok])
    assert np.all(np.isnan(out1[17])) and np.all(np.isnan(out2[17]))
    srv.close()


def test_submit_rejections(torch_dev):
    # the same argument rules as esom_embed, checked before anything is queued
    from paper_2201_00701_amd import esom
    from paper_2201_00701_amd.esom import Server
    X, L, l = _req(321, 500, 8, 50, 10)
    srv = Server(0, 0, 1)
    _say("case serve submit rejections")
    bad = [dict(k=2), dict(k=51), dict(boost=0.0), dict(boost=50.0), dict(cutoff=0.0),
           dict(cutoff=float("inf")), dict(gravity=-1.0), dict(gravity=float("nan")),
           dict(adjust=float("inf")), dict(mode=5), dict(candidates=51)]
    for kw in bad:
        p = {"k": 8, **kw}
        with pytest.raises(esom.EsomError) as e:
            srv.submit(L, l, X=X, **p)
        assert e.value.code == esom.ESOM_EINVAL, kw
    st = srv.stats()
    assert st["queued"] == 0 and st["completed"] == 0
    # and a valid request still runs
    info = srv.wait(srv.submit(L, l, k=8, X=X), 60000)
    np.testing.assert_array_equal(info["out"], _direct(torch_dev, X, L, l, 8, "fp32"))
    srv.close()
