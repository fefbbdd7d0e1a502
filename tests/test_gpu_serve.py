"""GPU tests of the serving loop (cfx_serve_*): results against the oracle,
the same bits alone and in a concurrent mix, resident factors and re-solves,
admission under a small HBM budget, and eviction."""
import time

import numpy as np
import pytest

import cfx_inputs as G
from oracle import oracle as O
from tests.gpu_util import say, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cfx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2010_05975_amd import cfx as m
    m.lib()
    return m


def make_requests(sizes, seed, cond=None):
    out = []
    for i, n in enumerate(sizes):
        if cond is None:
            A = G.normal_matrix(n, seed + i) + 2 * np.sqrt(n) * np.eye(n)
        else:
            A = G.householder_matrix(G.householder_spec(n, cond, seed + i))
        B = G.rhs(n, 1 + (i % 4), seed + 100 + i)
        out.append((A, B))
    return out


def solve_alone(srv, reqs):
    outs = []
    for A, B in reqs:
        dA, dB = to_dev(A), to_dev(B)
        dX = torch.zeros_like(dB)
        r = srv.wait(srv.submit(dA, dB, dX))
        outs.append((dX.cpu().numpy(), r))
    return outs


def solve_mix(srv, reqs):
    held = []
    for A, B in reqs:
        dA, dB = to_dev(A), to_dev(B)
        dX = torch.zeros_like(dB)
        held.append((srv.submit(dA, dB, dX), dX))
    out = []
    for t, dX in held:
        r = srv.wait(t)            # wait first: X is written by the server
        out.append((dX.cpu().numpy(), r))
    return out


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_serve_alone_equals_mix_and_oracle(cfx, prec):
    say(f"serve alone vs mix {prec}")
    sizes = [30, 700, 100, 1500, 64, 513, 300, 900, 17, 2048]
    reqs = make_requests(sizes, 40, cond=1e4 if prec != "fp64" else None)
    srv = cfx.Server(8 << 30, max_slots=4, precision=prec, v=128, leaves=4, tol=5e-15,
                     max_outer=20 if prec != "fp64" else 4, gmres_restart=30, gmres_tol=1e-6)
    try:
        alone = solve_alone(srv, reqs)
        mix = solve_mix(srv, reqs)
        stats = srv.stats()
    finally:
        srv.close()
    say(f"  stats {stats}")
    assert stats["batches"] >= 2            # the small requests went through batched launches
    for i, ((A, B), (xa, ra), (xm, rm)) in enumerate(zip(reqs, alone, mix)):
        tag = f"request {i} n={A.shape[0]}"
        assert ra["status"] == 0 and rm["status"] == 0, tag
        assert np.array_equal(xa, xm), tag
        assert ra["eta"] == rm["eta"], tag
        eta = O.eta(A, xa, B)
        assert eta <= 5e-15, (tag, eta, ra)
        assert abs(ra["eta"] - eta) <= 0.05 * eta + 1e-19, (tag, ra["eta"], eta)
        assert ra["batched"] == (1 if A.shape[0] <= 512 else 0), tag
        assert ra["t_submit"] <= ra["t_admit"] <= ra["t_start"] <= ra["t_done"], tag


def test_serve_lowp_falls_back_to_fp64(cfx):
    """BF16 factors of a cond-1e12 system cannot be refined to 5e-15 in three
    outer steps: the request refactors in FP64, reports it, still meets the
    target, and its resident factors stay FP64 for the re-solve.  A
    well-conditioned request of the same server needs no fallback."""
    say("serve low-precision fallback")
    srv = cfx.Server(4 << 30, max_slots=2, precision="bf16", v=128, leaves=4, tol=5e-15,
                     max_outer=3, gmres_restart=20, gmres_tol=1e-6)
    try:
        n = 700
        hard = G.householder_matrix(G.householder_spec(n, 1e12, 31))
        easy = G.householder_matrix(G.householder_spec(n, 1e2, 32))
        B = G.rhs(n, 2, 33)
        dH, dE = to_dev(hard), to_dev(easy)
        Xh = torch.zeros((n, 2), dtype=torch.float64, device="cuda")
        Xe = torch.zeros((n, 2), dtype=torch.float64, device="cuda")
        rh = srv.wait(srv.submit(dH, to_dev(B), Xh, keep_resident=True))
        re_ = srv.wait(srv.submit(dE, to_dev(B), Xe))
        say(f"  hard {rh}\n  easy {re_}")
        assert rh["status"] == 0 and rh["fallback"] == 1
        assert O.eta(hard, Xh.cpu().numpy(), B) <= 5e-15
        assert re_["status"] == 0 and re_["fallback"] == 0
        assert O.eta(easy, Xe.cpu().numpy(), B) <= 5e-15
        X2 = torch.zeros((n, 2), dtype=torch.float64, device="cuda")
        r2 = srv.wait(srv.submit(dH, to_dev(B), X2, kind=cfx.RESOLVE, factor_id=rh["factor_id"]))
        assert r2["resident_hit"] == 1 and r2["fallback"] == 0 and r2["status"] == 0
        assert O.eta(hard, X2.cpu().numpy(), B) <= 5e-15
    finally:
        srv.close()


def test_serve_resident_resolve_and_release(cfx):
    say("serve resident factors")
    srv = cfx.Server(4 << 30, max_slots=2, precision="fp64", v=64, leaves=4, max_outer=4)
    try:
        for n in (200, 800):
            A = G.normal_matrix(n, 5) + np.sqrt(n) * np.eye(n)
            dA = to_dev(A)
            B1, B2 = G.rhs(n, 2, 6), G.rhs(n, 3, 7)
            X1 = torch.zeros((n, 2), dtype=torch.float64, device="cuda")
            r1 = srv.wait(srv.submit(dA, to_dev(B1), X1, keep_resident=True))
            fid = r1["factor_id"]
            X2 = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
            r2 = srv.wait(srv.submit(dA, to_dev(B2), X2, kind=cfx.RESOLVE, factor_id=fid))
            say(f"  n={n} {r1} {r2}")
            assert r2["resident_hit"] == 1 and r2["factor_id"] == fid and r2["status"] == 0
            assert O.eta(A, X1.cpu().numpy(), B1) <= 5e-15
            assert O.eta(A, X2.cpu().numpy(), B2) <= 5e-15
            assert srv.release(fid) == 0
            X3 = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
            r3 = srv.wait(srv.submit(dA, to_dev(B2), X3, kind=cfx.RESOLVE, factor_id=fid))
            assert r3["resident_hit"] == 0 and r3["status"] == 0
            assert O.eta(A, X3.cpu().numpy(), B2) <= 5e-15
            if n > 512:
                # refactored by the same single-request path: the same bits
                assert np.array_equal(X3.cpu().numpy(), X2.cpu().numpy())
        st = srv.stats()
        assert st["resident_hits"] == 2 and st["resident_misses"] == 2
    finally:
        srv.close()


def test_serve_admission_under_budget(cfx):
    """An arena that holds one n = 1200 request at a time: requests run one
    after another, the peak stays within the budget, and a request that can
    never fit fails with CFX_ENOMEM instead of blocking the queue."""
    say("serve admission budget")
    n = 1200
    one = 2 * n * n * 8                 # factors plus workspace, with margin
    srv = cfx.Server(one, max_slots=4, precision="fp64", v=64, leaves=4, max_outer=2)
    try:
        reqs = make_requests([n, n, n], 70)
        big_A = to_dev(G.normal_matrix(3000, 1))
        big_B = to_dev(G.rhs(3000, 1, 2))
        big_X = torch.zeros_like(big_B)
        held = []
        for A, B in reqs:
            dA, dB = to_dev(A), to_dev(B)
            dX = torch.zeros_like(dB)
            held.append((srv.submit(dA, dB, dX), dX, A, B))
        tb = srv.submit(big_A, big_B, big_X)
        res = [(srv.wait(t), dX, A, B) for t, dX, A, B in held]
        rb = srv.wait(tb)
        st = srv.stats()
    finally:
        srv.close()
    say(f"  stats {st}; big {rb['status']}")
    assert rb["status"] == -1001
    assert st["bytes_peak"] <= one
    spans = sorted((r["t_start"], r["t_done"]) for r, *_ in res)
    for (s0, d0), (s1, d1) in zip(spans, spans[1:]):
        assert s1 >= d0 - 1e-6            # never two at once: the budget holds one
    for r, dX, A, B in res:
        assert r["status"] == 0
        assert O.eta(A, dX.cpu().numpy(), B) <= 5e-15


def test_serve_evicts_least_recently_used(cfx):
    say("serve eviction")
    n = 800
    per = n * n * 8 + 2 * n * 4 + 4096
    srv = cfx.Server(int(2.5 * per) + (2 << 20), max_slots=1, precision="fp64", v=64, leaves=4,
                     max_outer=2)
    try:
        ids = []
        mats = []
        for i in range(3):
            A = G.normal_matrix(n, 80 + i) + np.sqrt(n) * np.eye(n)
            B = G.rhs(n, 1, 90 + i)
            dA, dB = to_dev(A), to_dev(B)
            dX = torch.zeros_like(dB)
            r = srv.wait(srv.submit(dA, dB, dX, keep_resident=True))
            assert r["status"] == 0
            ids.append(r["factor_id"])
            mats.append((A, dA))
        st = srv.stats()
        assert st["evictions"] >= 1 and st["resident_factors"] <= 2
        # the oldest factor was evicted: a re-solve of it is a miss, the newest a hit
        A0, dA0 = mats[0]
        B = G.rhs(n, 1, 5)
        dX = torch.zeros((n, 1), dtype=torch.float64, device="cuda")
        r0 = srv.wait(srv.submit(dA0, to_dev(B), dX, kind=cfx.RESOLVE, factor_id=ids[0]))
        assert r0["resident_hit"] == 0 and O.eta(A0, dX.cpu().numpy(), B) <= 5e-15
        A2, dA2 = mats[2]
        r2 = srv.wait(srv.submit(dA2, to_dev(B), dX, kind=cfx.RESOLVE, factor_id=ids[2]))
        assert r2["resident_hit"] == 1
    finally:
        srv.close()


def test_lowp_routing_small_requests_take_fp64(cfx):
    """A BF16 server with lowp_min_n routes smaller requests to FP64
    factors: their results equal those of an FP64 server with the same
    refinement settings bit for bit, while requests at or above the
    threshold stay low precision (they need refinement steps)."""
    say("serve lowp routing")
    reqs = make_requests([600, 800, 1000], 61, cond=1e4)   # above the batched sizes
    kw = dict(v=64, leaves=4, tol=5e-15, max_outer=3, gmres_restart=20, gmres_tol=1e-6)
    srv64 = cfx.Server(256 << 20, max_slots=1, precision="fp64", **kw)
    srvr = cfx.Server(256 << 20, max_slots=1, precision="bf16", lowp_min_n=900, **kw)
    try:
        a = solve_alone(srv64, reqs)
        b = solve_alone(srvr, reqs)
    finally:
        srv64.close()
        srvr.close()
    for (xa, ra), (xb, rb), (A, B) in zip(a, b, reqs):
        assert ra["status"] == rb["status"] == 0
        assert O.eta(A, xb, B) <= 5e-15
    for i in (0, 1):                      # n < 900: FP64 factors on both servers
        assert np.array_equal(a[i][0], b[i][0])
        assert b[i][1]["fallback"] == 0 and b[i][1]["batched"] == 0
    assert b[2][1]["outer"] >= 1          # n = 1000: BF16 factors, refined
    assert a[2][1]["outer"] == 0
