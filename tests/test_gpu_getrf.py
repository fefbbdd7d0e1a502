"""GPU parity of the FP64 tournament-pivoted LU against the CPU oracle.

Every call goes through the C ABI (libcfx.so via the ctypes binding)."""
import numpy as np
import pytest

import cfx_inputs as G
from oracle import oracle as O
from tests.gpu_util import compare_panels, say, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cfx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2010_05975_amd import cfx as m
    m.lib()
    return m


# ---------------------------------------------------------------------------
# tournament alone
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("rows,vb,L", [(64, 8, 4), (512, 32, 4), (300, 32, 3), (1000, 16, 7),
                                       (2048, 64, 8), (4096, 256, 16), (1024, 256, 1),
                                       (700, 128, 5), (33, 32, 64), (8192, 256, 1),
                                       (6000, 256, 1), (4096, 128, 2), (2500, 256, 1)])
def test_tslu_matches_oracle(cfx, rows, vb, L):
    say(f"tslu rows={rows} vb={vb} L={L}")
    W = G.normal_matrix(rows, rows + vb)[:, :vb].copy()
    ref, margin = O.tslu(W, vb, L, row0=5)
    piv = cfx.tslu(to_dev(W), vb, L, row0=5).cpu().numpy()
    torch.cuda.synchronize()
    assert margin > 1e-10
    assert np.array_equal(piv, ref)


def test_tslu_ties_smallest_row(cfx):
    say("tslu ties")
    W = G.wilkinson_growth_matrix(96)[:, :32].copy()
    ref, _ = O.tslu(W, 32, 3)
    piv = cfx.tslu(to_dev(W), 32, 3).cpu().numpy()
    assert np.array_equal(piv, ref)
    assert np.array_equal(piv, np.arange(32))


# ---------------------------------------------------------------------------
# full factorisation
# ---------------------------------------------------------------------------

def run_getrf(cfx, A, v, L, lookahead=0, prec="fp64"):
    dA = to_dev(A)
    ipiv, info = cfx.getrf(dA, v=v, leaves=L, lookahead=lookahead, precision=prec)
    torch.cuda.synchronize()
    return dA.cpu().numpy(), ipiv.cpu().numpy(), int(info.cpu()[0])


def lu_tolerance(ref_LU, n):
    # forward error of each factor entry: about n * eps * (|L||U|) with
    # growth; 1e-9 relative to max|U| leaves room for pivot-order rounding.
    return 1e-9 * max(1.0, float(np.abs(ref_LU).max()))


@pytest.mark.parametrize("gen,n,v,L", [
    ("uniform", 512, 32, 4),     # the small single-matrix case
    ("normal", 300, 32, 3),      # ragged last panel
    ("normal", 257, 16, 6),
    ("uniform", 100, 128, 4),    # n < v
    ("normal", 1, 32, 4),
    ("normal", 1024, 64, 8),
    ("normal", 2048, 256, 4),
    ("normal", 777, 256, 2),
    ("normal", 4096, 256, 1),    # one 4096-row leaf (16 rows per thread)
    ("normal", 4096, 256, 2),    # 2048-row leaves
    ("normal", 3000, 128, 3),    # 1000-row leaves, ragged
    ("normal", 6000, 256, 8),    # the bench's leaf count, 750-row leaves
])
@pytest.mark.parametrize("lookahead", [0, 1])
def test_getrf_matches_oracle(cfx, gen, n, v, L, lookahead):
    say(f"getrf {gen} n={n} v={v} L={L} lookahead={lookahead}")
    A = getattr(G, f"{gen}_matrix")(n, 17)
    ref = O.getrf(A, v, L)
    LU, ipiv, info = run_getrf(cfx, A, v, L, lookahead)
    assert info == ref.info == 0
    compared = compare_panels(ipiv, ref.ipiv, ref.margins, v)
    say(f"  panels compared {compared}/{len(ref.margins)}")
    assert O.lu_residual(A, LU, ipiv) <= 1e-12
    if compared == len(ref.margins):
        np.testing.assert_allclose(LU, ref.LU, rtol=0, atol=lu_tolerance(ref.LU, n))


@pytest.mark.parametrize("n,v,L", [(64, 8, 4), (200, 32, 3), (96, 32, 1)])
def test_getrf_wilkinson_exact(cfx, n, v, L):
    say(f"wilkinson n={n}")
    A = G.wilkinson_growth_matrix(n)
    LU, ipiv, info = run_getrf(cfx, A, v, L)
    ref = O.getrf(A, v, L)
    assert np.array_equal(ipiv, np.arange(n))
    assert np.array_equal(LU, ref.LU)


@pytest.mark.parametrize("n,v,L", [(64, 8, 4), (64, 16, 3), (50, 7, 5)])
def test_getrf_dd_exact(cfx, n, v, L):
    say(f"dd n={n} v={v}")
    L0, U0 = G.dyadic_dd_factors(n, 1)
    A = L0 @ U0
    LU, ipiv, info = run_getrf(cfx, A, v, L)
    assert np.array_equal(ipiv, np.arange(n))
    assert np.array_equal(np.tril(LU, -1) + np.eye(n), L0)
    assert np.array_equal(np.triu(LU), U0)


@pytest.mark.parametrize("lookahead", [0, 1])
def test_getrf_zero_column_info(cfx, lookahead):
    say(f"zero column lookahead={lookahead}")
    n = 80
    A = G.normal_matrix(n, 4)
    A[:, 37] = 0.0
    LU, ipiv, info = run_getrf(cfx, A, 16, 3, lookahead)
    ref = O.getrf(A, 16, 3)
    assert info == ref.info == 38
    assert np.array_equal(ipiv, ref.ipiv)
    np.testing.assert_allclose(LU, ref.LU, rtol=0, atol=1e-9 * np.abs(ref.LU).max())


def test_getrf_empty(cfx):
    say("empty")
    A = torch.zeros((0, 0), dtype=torch.float64, device="cuda")
    ipiv, info = cfx.getrf(A, v=32, leaves=4)
    torch.cuda.synchronize()
    assert int(info.cpu()[0]) == 0


# ---------------------------------------------------------------------------
# solve
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,nrhs,v,L", [(512, 1, 32, 4), (300, 5, 32, 3), (1000, 64, 64, 4),
                                        (600, 1, 256, 2), (1, 1, 32, 4), (63, 2, 16, 2),
                                        (64, 1, 16, 2), (65, 17, 16, 2), (127, 16, 32, 3),
                                        (128, 1, 32, 3), (129, 64, 32, 3), (257, 3, 64, 2),
                                        (2000, 1, 128, 8), (4097, 1, 256, 4), (1, 1, 1, 1)])
def test_getrs_matches_oracle(cfx, n, nrhs, v, L):
    say(f"getrs n={n} nrhs={nrhs}")
    A = G.normal_matrix(n, 3)
    B = G.rhs(n, nrhs, 4)
    ref = O.getrf(A, v, L)
    Xref = O.getrs(ref.LU, ref.ipiv, B)
    dA = to_dev(A)
    ipiv, info = cfx.getrf(dA, v=v, leaves=L)
    dB = to_dev(B)
    cfx.getrs(dA, ipiv, dB)
    X = dB.cpu().numpy()
    # A direct FP64 solve's backward error is a small multiple of n*u (not the
    # 5e-15 refinement target); it must stay within 4x of the oracle's own.
    eta_ref = O.eta(A, Xref, B)
    assert O.eta(A, X, B) <= max(4 * eta_ref, 1e-15)
    np.testing.assert_allclose(X, Xref, rtol=1e-8, atol=1e-8 * np.abs(Xref).max())


@pytest.mark.parametrize("kind", ["chain", "near", "uniform", "invalid"])
@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 36864, 36865])
def test_getrs_interchanges_exact(cfx, kind, n):
    """With unit factors (LU = I) getrs returns P B, so the composed
    interchanges are compared exactly with the sequential definition, for
    interchange runs that all share rows ("chain"), often do ("near") or
    rarely do ("uniform"); entries outside [i, n) are no interchange.
    n = 36864 is the largest order of the LDS index array, 36865 the first
    beyond it."""
    nrhs = 1 if kind in ("chain", "uniform") else 2
    say(f"getrs interchanges {kind} n={n} nrhs={nrhs}")
    ipiv = G.ipiv_pattern(kind, n, 21)
    i = np.arange(n)
    perm = O.ipiv_to_perm(np.where((ipiv >= i) & (ipiv < n), ipiv, i))
    B = G.rhs(n, nrhs, 22)
    dLU = torch.eye(n, dtype=torch.float64, device="cuda")
    dB = to_dev(B)
    cfx.getrs(dLU, torch.from_numpy(ipiv).cuda(), dB)
    X = dB.cpu().numpy()
    del dLU
    assert np.array_equal(X, B[perm])


@pytest.mark.parametrize("n,v,L", [(1500, 128, 4), (3000, 256, 8)])
def test_getrf_lookahead_bitwise_equal(cfx, n, v, L):
    """Lookahead only reorders independent launches: the factors are
    bitwise the same as without it."""
    say(f"lookahead bitwise n={n} v={v} L={L}")
    A = G.normal_matrix(n, 8)
    a = run_getrf(cfx, A, v, L, 0)
    b = run_getrf(cfx, A, v, L, 1)
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[0], b[0])


def test_overlap_tuning_rejects_invalid_values(cfx):
    """cfx_set_overlap_tuning: -2 for a workgroup bound below -1 or in
    1..7, -3 for chunk_cols < 0, -4 for one_stream outside {0, 1}; a
    rejected call leaves the settings unchanged."""
    h = cfx.Handle()
    try:
        cfx.set_overlap_tuning(8, 256, 1, handle=h)
        for args, code in [((-2, 512, 0), -2), ((1, 512, 0), -2), ((7, 512, 0), -2),
                           ((0, -1, 0), -3), ((0, 512, 2), -4)]:
            with pytest.raises(cfx.CfxError) as e:
                cfx.set_overlap_tuning(*args, handle=h)
            assert e.value.code == code, args
            assert cfx.overlap_tuning(handle=h) == (8, 256, 1)
        cfx.set_overlap_tuning(-1, 0, 0, handle=h)
        assert cfx.overlap_tuning(handle=h) == (-1, 0, 0)
    finally:
        h.close()


def test_reserved_cus_settings(cfx):
    """cfx_set_reserved_cus: default 32 on a 256-CU device, 0..CUs/4
    accepted (0 = the caller's stream), -2 otherwise with the setting
    unchanged."""
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    h = cfx.Handle()
    try:
        assert cfx.reserved_cus(handle=h) == min(32, ncu // 4)
        for bad in (-1, ncu // 4 + 1, 10000):
            with pytest.raises(cfx.CfxError) as e:
                cfx.set_reserved_cus(bad, handle=h)
            assert e.value.code == -2
            assert cfx.reserved_cus(handle=h) == min(32, ncu // 4)
        for good in (0, 8, ncu // 4):
            cfx.set_reserved_cus(good, handle=h)
            assert cfx.reserved_cus(handle=h) == good
    finally:
        h.close()


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_reserved_cus_bitwise_equal(cfx, prec):
    """The rest of each update on the CU-masked stream (0, 8 or 32
    reserved compute units, automatic or fixed chunks, interchanged or
    masked rows) changes scheduling only: the factors are bitwise those of
    the plain schedule on the caller's stream."""
    n, v, L = 2304, 128, 4
    say(f"reserved cus bitwise {prec} n={n}")
    A = G.normal_matrix(n, 21)
    ref = run_getrf(cfx, A, v, L, 0, prec=prec)
    for cus, chunk, masked in [(0, 0, False), (8, 0, False), (32, 0, False), (32, 300, False), (32, 0, True)]:
        h = cfx.Handle()
        try:
            cfx.set_reserved_cus(cus, handle=h)
            cfx.set_overlap_tuning(-1, chunk, 0, handle=h)
            dA = to_dev(A)
            if masked:
                ipiv, rowmap, info = cfx.getrf_masked(dA, v=v, leaves=L, precision=prec, lookahead=1, handle=h)
            else:
                ipiv, info = cfx.getrf(dA, v=v, leaves=L, precision=prec, lookahead=1, handle=h)
            torch.cuda.synchronize()
        finally:
            h.close()
        LU = dA.cpu().numpy()
        if masked:
            LU = LU[rowmap.cpu().numpy()[:n]]
        assert int(info.cpu()[0]) == ref[2]
        assert np.array_equal(ipiv.cpu().numpy()[:n], ref[1][:n]), (cus, chunk, masked)
        assert np.array_equal(LU, ref[0]), (cus, chunk, masked)


@pytest.mark.parametrize("masked", [False, True])
def test_full_trsm_rows_bitwise_equal(cfx, masked):
    """All of U12 solved in the first launch (threshold 0) or split between
    the first launch and the rest of the update (threshold above the matrix)
    is scheduling only: the same pivots and factors bit for bit."""
    n, v, L = 2304, 128, 4
    say(f"full-U12 threshold bitwise masked={masked}")
    A = G.normal_matrix(n, 23)
    got = []
    for rows in (1 << 30, 0, 1000):
        h = cfx.Handle()
        try:
            cfx.set_full_trsm_rows(rows, handle=h)
            assert cfx.full_trsm_rows(handle=h) == rows
            dA = to_dev(A)
            if masked:
                ipiv, rowmap, info = cfx.getrf_masked(dA, v=v, leaves=L, lookahead=1, handle=h)
            else:
                ipiv, info = cfx.getrf(dA, v=v, leaves=L, lookahead=1, handle=h)
            torch.cuda.synchronize()
        finally:
            h.close()
        LU = dA.cpu().numpy()
        if masked:
            LU = LU[rowmap.cpu().numpy()[:n]]
        got.append((LU, ipiv.cpu().numpy()[:n], int(info.cpu()[0])))
    for LU, ipiv, info in got[1:]:
        assert info == got[0][2]
        assert np.array_equal(ipiv, got[0][1])
        assert np.array_equal(LU, got[0][0])
    ref = O.getrf(A, v, L)
    compare_panels(got[0][1], ref.ipiv, ref.margins, v)


@pytest.mark.parametrize("n,wgs,chunk", [(2100, 8, 64), (2100, 12, 300), (2100, 40, 4096), (2048, 8, 256),
                                         (2048, 24, 4096)])
def test_getrf_bounded_schur_grid_bitwise_equal(cfx, n, wgs, chunk):
    """The overlapped Schur launches with a bounded, persistent grid (few
    workgroups walking many tiles, in narrow or wide column chunks, ragged
    or whole tiles) change scheduling only: the factors are bitwise those of
    the plain schedule."""
    v, L = 128, 4
    say(f"bounded schur grid wgs={wgs} chunk={chunk} n={n}")
    A = G.normal_matrix(n, 12)
    ref = run_getrf(cfx, A, v, L, 0)
    h = cfx.Handle()
    try:
        assert cfx.overlap_tuning(handle=h) == (-1, 0, 0)     # the defaults
        one = 1 if wgs == 12 else 0         # one case on the caller's stream only
        cfx.set_overlap_tuning(wgs, chunk, one, handle=h)
        assert cfx.overlap_tuning(handle=h) == (wgs, chunk, one)
        dA = to_dev(A)
        ipiv, info = cfx.getrf(dA, v=v, leaves=L, lookahead=1, handle=h)
        torch.cuda.synchronize()
    finally:
        h.close()
    assert int(info.cpu()[0]) == ref[2]
    assert np.array_equal(ipiv.cpu().numpy(), ref[1])
    assert np.array_equal(dA.cpu().numpy(), ref[0])


def test_getrs_one_rhs_repeat_is_deterministic(cfx):
    """The one-launch-per-triangle solve (blocks applying each other's
    results as they appear) gives the same bits on every call, and a column
    of a multi-column solve (a different code path) agrees to rounding."""
    n, v, L = 3000, 128, 4
    say(f"getrs determinism n={n}")
    A = G.normal_matrix(n, 14)
    dA = to_dev(A)
    ipiv, info = cfx.getrf(dA, v=v, leaves=L)
    B = G.rhs(n, 2, 15)
    outs = []
    for rep in range(3):
        dB = to_dev(B[:, :1].copy())
        cfx.getrs(dA, ipiv, dB)
        torch.cuda.synchronize()
        outs.append(dB.cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    dB2 = to_dev(B)
    cfx.getrs(dA, ipiv, dB2)
    X2 = dB2.cpu().numpy()
    np.testing.assert_allclose(outs[0][:, 0], X2[:, 0], rtol=0, atol=1e-10 * np.abs(X2).max())
    assert O.eta(A, outs[0], B[:, :1]) <= 1e-14


@pytest.mark.parametrize("kind", ["zeros", "zero_pivot"])
def test_getrs_one_rhs_degenerate_values(cfx, kind):
    """The one-right-hand-side solve's fast substitution lets a row that is
    already final take v - 0 * x; when a result of a block is zero or not
    finite the block is solved again keeping each row's value at its own
    step.  Exact zeros in the solution, and a zero on U's diagonal (the rows
    solved before it must stay finite and correct), take that path; both
    are compared with the oracle.  Factors: unit L = I, U upper triangular,
    no interchanges."""
    n = 300
    say(f"getrs degenerate values {kind} n={n}")
    rng = np.random.default_rng(91)
    LU = np.triu(rng.standard_normal((n, n))) + np.diag(np.full(n, 4.0))
    ipiv = np.arange(n, dtype=np.int32)
    if kind == "zeros":
        x = rng.standard_normal(n)
        x[n // 2:] = 0.0
        b = np.triu(LU) @ x            # rows n/2.. of b are exactly zero
    else:
        LU[n // 2, n // 2] = 0.0
        b = rng.standard_normal(n)
    B = b.reshape(n, 1)
    Xref = O.getrs(LU, ipiv, B)
    dB = to_dev(B)
    cfx.getrs(to_dev(LU), torch.from_numpy(ipiv).cuda(), dB)
    assert cfx.getrs_check() == 0
    X = dB.cpu().numpy()
    fin = np.isfinite(Xref)
    assert np.array_equal(fin, np.isfinite(X))
    if kind == "zero_pivot":
        assert fin[n // 2 + 1:].all() and not fin[: n // 2 + 1].any()
    np.testing.assert_allclose(X[fin], Xref[fin], rtol=1e-10, atol=1e-12 * np.abs(Xref[fin]).max())
    if kind == "zeros":
        assert np.all(X[n // 2:] == 0.0)


def _golden(n):
    import os
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    import make_c2_golden as MG
    if not os.path.exists(MG.path(n)):
        pytest.fail(f"stored oracle results for N={n} are missing: run tests/golden/make_c2_golden.py {n}")
    return MG, MG.load(n)


def gpu_frob_residual(A0, LU, perm, block=2048):
    """||P A - L U||_F / ||A||_F on the GPU with torch's own FP64 matrix
    products (an independent checker: none of the library's kernels), block
    row by block row; A0 and LU are device tensors, perm a host index array."""
    n = A0.shape[0]
    dperm = torch.from_numpy(np.ascontiguousarray(perm, dtype=np.int64)).cuda()
    U = torch.triu(LU)
    num = torch.zeros((), dtype=torch.float64, device=A0.device)
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        Lb = torch.tril(LU[r0:r1, :r1], diagonal=r0 - 1)
        idx = torch.arange(r1 - r0, device=A0.device)
        Lb[idx, idx + r0] = 1.0
        D = A0[dperm[r0:r1]] - Lb @ U[:r1]
        num += (D * D).sum()
    del U
    return float(torch.sqrt(num) / torch.linalg.norm(A0))


@pytest.mark.parametrize("n", [16384, 32768])
def test_getrf_full_size_against_stored_oracle(cfx, n):
    """The plain FP64 workload at full size (A ~ N(0,1) seed 0, v = 256,
    L = 8 with leaves of at least 4096 rows, lookahead, as the bench runs
    it): every panel's pivots bit for bit
    against the oracle's whole factorisation (stored by
    tests/golden/make_c2_golden.py) up to the first panel whose oracle margin
    is <= 1e-10, and ||P A - L U||_F / ||A||_F <= 1e-12 computed on the GPU
    by an independent checker."""
    v, L = 256, 8
    MG, gold = _golden(n)
    say(f"full size n={n}: generating")
    A = G.normal_matrix(n, int(gold["seed"]))
    assert MG.digest(A) == str(gold["digest"]), "the generator no longer gives the stored input"
    A0 = to_dev(A)
    del A
    dA = A0.clone()
    R = int(gold["min_leaf_rows"]) if "min_leaf_rows" in gold else 0
    ipiv, info = cfx.getrf(dA, v=v, leaves=L, lookahead=1, min_leaf_rows=R)
    torch.cuda.synchronize()
    piv = ipiv.cpu().numpy()
    assert int(info.cpu()[0]) == int(gold["info"]) == 0
    assert np.all(piv >= np.arange(n)) and np.all(piv < n)
    npan = compare_panels(piv, gold["ipiv"], gold["margins"], v)
    say(f"  pivots equal on {npan} of {len(gold['margins'])} panels "
        f"(min oracle margin {gold['margins'].min():.2e})")
    assert npan == len(gold["margins"]) or gold["margins"][npan] <= 1e-10
    say("  residual on the GPU")
    res = gpu_frob_residual(A0, dA, O.ipiv_to_perm(piv))
    say(f"  ||PA-LU||_F/||A||_F = {res:.3e} (oracle's own factors: {float(gold['residual']):.3e})")
    assert res <= 1e-12


@pytest.mark.parametrize("n,v,L,la", [(2048, 256, 8, 1), (3000, 128, 4, 0), (700, 64, 3, 1), (5000, 256, 16, 1)])
def test_fused_tournament_nodes_bitwise_equal(cfx, n, v, L, la):
    """Nodes of at most 512 rows run as one launch each (pivot steps and the
    node's own updates in one workgroup) or as two launches per column
    block: a scheduling choice only, so the factors are equal bit for bit."""
    say(f"fused tournament nodes n={n} v={v} L={L} la={la}")
    A = G.normal_matrix(n, 900 + n)
    out = []
    for rows in (512, 0):
        h = cfx.Handle()
        try:
            cfx.set_tournament_fusion(rows, handle=h)
            assert cfx.tournament_fusion(handle=h) == rows
            dA = to_dev(A)
            ipiv, info = cfx.getrf(dA, v=v, leaves=L, lookahead=la, handle=h)
            torch.cuda.synchronize()
            out.append((dA.cpu().numpy(), ipiv.cpu().numpy(), int(info.cpu()[0])))
        finally:
            h.close()
    assert out[0][2] == out[1][2] == 0
    assert np.array_equal(out[0][1], out[1][1])
    assert np.array_equal(out[0][0], out[1][0])
    ref = O.getrf(A, v, L)
    assert compare_panels(out[0][1][:n], ref.ipiv, ref.margins, v) == len(ref.margins)


@pytest.mark.parametrize("n,v,L,R,la", [(2048, 128, 8, 512, 1), (1500, 100, 5, 300, 0), (3000, 256, 8, 1024, 1),
                                        (777, 64, 4, 200, 1)])
def test_min_leaf_rows_matches_oracle(cfx, n, v, L, R, la):
    """Leaves of at least R rows (min(L, max(1, ceil(r / R))) leaves for a
    panel of r rows): pivots bit for bit against the oracle with the same
    rule panel by panel (margin rule), factors within rounding, residual
    <= 1e-12; the masked factorisation gives the same factors through its
    row map."""
    say(f"min leaf rows n={n} v={v} L={L} R={R} la={la}")
    A = G.normal_matrix(n, 1300 + n)
    ref = O.getrf(A, v, L, min_leaf_rows=R)
    dA = to_dev(A)
    ipiv, info = cfx.getrf(dA, v=v, leaves=L, lookahead=la, min_leaf_rows=R)
    torch.cuda.synchronize()
    LU, piv = dA.cpu().numpy(), ipiv.cpu().numpy()[:n]
    assert int(info.cpu()[0]) == ref.info == 0
    npan = compare_panels(piv, ref.ipiv, ref.margins, v)
    assert npan == len(ref.margins)
    np.testing.assert_allclose(LU, ref.LU, rtol=0, atol=lu_tolerance(ref.LU, n))
    assert O.lu_residual(A, LU, piv) <= 1e-12
    dM = to_dev(A)
    ipm, rowmap, infom = cfx.getrf_masked(dM, v=v, leaves=L, lookahead=la, min_leaf_rows=R)
    torch.cuda.synchronize()
    assert np.array_equal(ipm.cpu().numpy()[:n], piv)
    assert np.array_equal(dM.cpu().numpy()[rowmap.cpu().numpy()[:n]], LU)
