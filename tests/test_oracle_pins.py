"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test checks the oracle's TP(v, L) LU (the compute steps of Alg. 1 with
the tournament pivoting of Sec. 7.3) against something independent:

* the greedy max-|det| characterisation of partial pivoting, evaluated in
  exact rational arithmetic (a GEPP node's j-th pivot maximises the
  (j+1)-minor over the rows not yet chosen);
* a tournament whose nodes are LAPACK's dgetrf (scipy), i.e. a library GEPP;
* special cases that reduce to textbook results (v = 1 and L = 1 are partial
  pivoting; the Wilkinson growth matrix; exactly representable diagonally
  dominant factors; Leibniz determinants);
* the statement counts of the in-place LU program (Sec. 6, S1 and S2).
"""
from fractions import Fraction
import itertools
import os
import subprocess
import sys

import numpy as np
import pytest
import scipy.linalg as sl

import cfx_inputs as G
from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


# ---------------------------------------------------------------------------
# Independent helpers (exact rationals, LAPACK)
# ---------------------------------------------------------------------------

def frac_det(M):
    """Exact determinant of a square list-of-lists of Fractions (elimination)."""
    M = [row[:] for row in M]
    n = len(M)
    det = Fraction(1)
    for j in range(n):
        p = next((i for i in range(j, n) if M[i][j] != 0), None)
        if p is None:
            return Fraction(0)
        if p != j:
            M[j], M[p] = M[p], M[j]
            det = -det
        det *= M[j][j]
        for i in range(j + 1, n):
            f = M[i][j] / M[j][j]
            if f:
                for c in range(j, n):
                    M[i][c] -= f * M[j][c]
    return det


def leibniz_det(M):
    n = len(M)
    total = Fraction(0)
    for perm in itertools.permutations(range(n)):
        inv = sum(1 for a in range(n) for b in range(a + 1, n) if perm[a] > perm[b])
        prod = Fraction(1)
        for i in range(n):
            prod *= M[i][perm[i]]
        total += -prod if inv % 2 else prod
    return total


def greedy_det_selection(block, gids, vb):
    """Rows chosen by partial pivoting, characterised by minors.

    After rows P are chosen for columns 0..j-1, the Schur-complement entry of
    row r in column j equals det(B[P+[r], :j+1]) / det(B[P, :j]); the
    denominator is common, so the pivot maximises |det(B[P+[r], :j+1])|.
    Ties go to the smallest global row index.  Returns (selection, margins).
    """
    B = [[Fraction(float(x)) for x in row] for row in block]
    rows = len(B)
    chosen, margins = [], []
    for j in range(min(vb, rows)):
        cands = [r for r in range(rows) if r not in chosen]
        vals = []
        for r in cands:
            sub = [B[q][: j + 1] for q in chosen + [r]]
            vals.append(abs(frac_det(sub)))
        best = max(vals)
        pick = min((gids[r] for r, v in zip(cands, vals) if v == best))
        r_pick = gids.index(pick)
        others = [v for r, v in zip(cands, vals) if r != r_pick]
        if not others:
            margins.append(1.0)
        elif best == 0:
            margins.append(0.0)
        else:
            margins.append(float((best - max(others)) / best))
        chosen.append(r_pick)
    return [gids[r] for r in chosen], margins


def lapack_select(block, vb):
    """GEPP selection of a block by LAPACK dgetrf (selection order, local idx)."""
    lu, piv, info = sl.lapack.dgetrf(np.array(block, dtype=np.float64))
    perm = np.arange(block.shape[0])
    for j, p in enumerate(piv):
        perm[j], perm[p] = perm[p], perm[j]
    return perm[: min(vb, block.shape[0])]


def lapack_tournament(W, vb, L):
    """TP(vb, L) with every node a LAPACK GEPP; returns root pivots (local)."""
    rows = W.shape[0]
    h = max(vb, -(-rows // L))
    nodes = []
    for r0 in range(0, rows, h):
        idx = np.arange(r0, min(r0 + h, rows))
        nodes.append(idx[lapack_select(W[idx, :vb], vb)])
    while len(nodes) > 1:
        nxt = []
        for a in range(0, len(nodes), 2):
            if a + 1 == len(nodes):
                nxt.append(nodes[a])
                continue
            idx = np.concatenate([nodes[a], nodes[a + 1]])
            nxt.append(idx[lapack_select(W[idx, :vb], vb)])
        nodes = nxt
    return nodes[0]


def lapack_ipiv(A):
    lu, piv, info = sl.lapack.dgetrf(A)
    return lu, piv.astype(np.int32)


# ---------------------------------------------------------------------------
# Node and tree semantics
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("rows,vb", [(5, 3), (7, 4), (9, 2), (6, 6)])
def test_gepp_node_equals_greedy_minor_rule(seed, rows, vb):
    """One leaf (L = 1): the oracle's selection is the max-minor greedy rule."""
    W = G.normal_matrix(max(rows, vb), seed)[:rows, :vb]
    piv, margin = O.tslu(W, vb, 1)
    sel, margins = greedy_det_selection(W, list(range(rows)), vb)
    assert list(piv) == sel
    assert margin == pytest.approx(min(margins), rel=1e-9, abs=1e-15)


def test_gepp_tie_break_smallest_row():
    """Exact ties in the first column go to the smallest row index, and
    later ties (after exact dyadic elimination) as well."""
    W = np.array([[1.0, 0.5], [-1.0, 0.5], [1.0, -0.5], [0.5, 2.0]])
    piv, margin = O.tslu(W, 2, 1)
    sel, _ = greedy_det_selection(W, [0, 1, 2, 3], 2)
    assert list(piv) == sel == [0, 3]
    assert margin == 0.0
    # same rows behind a tournament of two leaves: leaf0 {0,1} -> [0,1],
    # leaf1 {2,3} -> [2,3]; the merge sees rows [0,1,2,3] in that order.
    piv2, _ = O.tslu(W, 2, 2)
    assert list(piv2) == [0, 3]


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("rows,vb,L", [(64, 4, 4), (100, 8, 3), (257, 16, 5),
                                       (96, 32, 8), (1000, 32, 7), (40, 8, 64)])
def test_tournament_equals_lapack_noded_tree(seed, rows, vb, L):
    """The full tree (leaf height, pairing, promotion, current-step values)
    against the same tree with LAPACK dgetrf at every node."""
    W = G.normal_matrix(rows, seed)[:, :vb].copy()
    piv, margin = O.tslu(W, vb, L)
    ref = lapack_tournament(W, vb, L)
    assert margin > 1e-12
    assert list(piv) == list(ref)


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("rows,vb,L", [(12, 3, 2), (10, 2, 3), (16, 4, 4)])
def test_tournament_equals_greedy_rule_per_node(seed, rows, vb, L):
    """Tiny tournaments where every node is checked with exact minors."""
    W = G.uniform_matrix(rows, seed)[:, :vb].copy()
    piv, margin = O.tslu(W, vb, L)
    h = max(vb, -(-rows // L))
    nodes = []
    allm = []
    for r0 in range(0, rows, h):
        g = list(range(r0, min(r0 + h, rows)))
        s, m = greedy_det_selection(W[g], g, vb)
        nodes.append(s)
        allm += m
    while len(nodes) > 1:
        nxt = []
        for a in range(0, len(nodes), 2):
            if a + 1 == len(nodes):
                nxt.append(nodes[a])
                continue
            g = nodes[a] + nodes[a + 1]
            s, m = greedy_det_selection(W[g], g, vb)
            nxt.append(s)
            allm += m
        nodes = nxt
    assert list(piv) == nodes[0]
    assert margin == pytest.approx(min(allm), rel=1e-9, abs=1e-15)


# ---------------------------------------------------------------------------
# Whole factorisation: special cases that reduce to textbook results
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,L", [(50, 1), (50, 4), (133, 7)])
def test_v1_is_partial_pivoting(n, L):
    A = G.normal_matrix(n, 11)
    f = O.getrf(A, 1, L)
    lu, piv = lapack_ipiv(A)
    assert np.array_equal(f.ipiv, piv)
    np.testing.assert_allclose(f.LU, lu, rtol=0, atol=1e-12)


@pytest.mark.parametrize("n,v", [(64, 4), (200, 32), (512, 32), (300, 64)])
def test_single_leaf_is_gepp(n, v):
    A = G.uniform_matrix(n, 5)
    f = O.getrf(A, v, 1)
    lu, piv = lapack_ipiv(A)
    assert np.array_equal(f.ipiv, piv)
    np.testing.assert_allclose(f.LU, lu, rtol=0, atol=1e-11)
    assert np.abs(np.tril(f.LU, -1)).max() <= 1.0


@pytest.mark.parametrize("n,v", [(8, 8), (20, 32), (33, 64)])
def test_n_at_most_v_is_one_gepp(n, v):
    A = G.normal_matrix(n, 3)
    f = O.getrf(A, v, 4)
    lu, piv = lapack_ipiv(A)
    assert np.array_equal(f.ipiv, piv)
    np.testing.assert_allclose(f.LU, lu, rtol=0, atol=1e-12)


@pytest.mark.parametrize("n", [8, 37, 64, 200])
@pytest.mark.parametrize("v,L", [(1, 1), (4, 3), (8, 2), (32, 4)])
def test_wilkinson_closed_form(n, v, L):
    """Every column is an exact tie; smallest-index ties mean no interchange.
    Closed form: L_ij = -1 (i > j), U = I except U[i, n-1] = 2^i."""
    A = G.wilkinson_growth_matrix(n)
    f = O.getrf(A, v, L)
    assert np.array_equal(f.ipiv, np.arange(n))
    Lx = np.tril(-np.ones((n, n)), -1) + np.eye(n)
    Ux = np.eye(n)
    Ux[:, -1] = 2.0 ** np.arange(n)
    Lf, Uf = O.unpack(f.LU)
    assert np.array_equal(Lf, Lx)
    assert np.array_equal(Uf, Ux)
    assert f.margins.min() == 0.0


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("n,v,L", [(64, 8, 4), (64, 16, 3), (50, 7, 5), (64, 64, 1)])
def test_dd_dyadic_exact_factors(seed, n, v, L):
    """A = L0 U0 strictly column diagonally dominant with exact arithmetic:
    no interchanges for any (v, L) and bit-exact factors."""
    L0, U0 = G.dyadic_dd_factors(n, seed)
    A = L0 @ U0
    assert np.all(2 * np.abs(np.diag(A)) > np.abs(A).sum(axis=0))
    f = O.getrf(A, v, L)
    assert np.array_equal(f.ipiv, np.arange(n))
    Lf, Uf = O.unpack(f.LU)
    assert np.array_equal(Lf, L0)
    assert np.array_equal(Uf, U0)


@pytest.mark.parametrize("seed", range(3))
def test_permuted_dd_recovers_permutation(seed):
    n = 48
    L0, U0 = G.dyadic_dd_factors(n, seed)
    A = L0 @ U0
    pi = np.random.default_rng(seed).permutation(n)
    f = O.getrf(A[pi], 8, 1)
    assert np.array_equal(O.ipiv_to_perm(f.ipiv), np.argsort(pi))
    Lf, Uf = O.unpack(f.LU)
    assert np.array_equal(Lf, L0)
    assert np.array_equal(Uf, U0)


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("n,v,L", [(5, 2, 2), (6, 2, 3), (7, 3, 2), (4, 1, 4)])
def test_det_matches_leibniz(seed, n, v, L):
    A = np.random.default_rng(seed).integers(-4, 5, size=(n, n)).astype(np.float64)
    exact = leibniz_det([[Fraction(int(x)) for x in r] for r in A])
    f = O.getrf(A, v, L)
    d = O.ipiv_sign(f.ipiv) * np.prod(np.diag(f.LU))
    if exact == 0:
        assert abs(d) <= 1e-9 * np.prod(np.abs(A).sum(axis=1))
    else:
        assert d == pytest.approx(float(exact), rel=1e-10)


@pytest.mark.parametrize("gen,n,v,L", [("uniform", 512, 32, 4), ("normal", 300, 32, 3),
                                       ("normal", 257, 16, 6), ("uniform", 100, 128, 4)])
def test_residual_and_structure(gen, n, v, L):
    A = getattr(G, f"{gen}_matrix")(n, 1)
    f = O.getrf(A, v, L)
    assert f.info == 0
    assert O.lu_residual(A, f.LU, f.ipiv) <= 1e-12
    # ipiv is LAPACK-style: ipiv[i] >= i
    assert np.all(f.ipiv >= np.arange(n))
    # The root's own elimination bounds its multipliers: |L00| <= 1.
    for k in range(0, n, v):
        vb = min(v, n - k)
        assert np.abs(np.tril(f.LU[k:k + vb, k:k + vb], -1)).max(initial=0) <= 1.0


@pytest.mark.parametrize("n,v", [(1, 1), (2, 1), (10, 3), (100, 32), (257, 16), (512, 32)])
def test_statement_counts(n, v):
    """S1 runs N(N-1)/2 times and S2 sum_k (N-k-1)^2 times (Sec. 6); the
    leading term of the latter is the paper's N^3/3."""
    A = G.normal_matrix(n, 2)
    f = O.getrf(A, v, 3)
    div, ms = f.counters
    assert div == n * (n - 1) // 2
    assert ms == (n - 1) * n * (2 * n - 1) // 6
    if n >= 100:
        paper_vs2 = n ** 3 / 3 - n ** 2 + 2 * n / 3
        assert abs(ms / paper_vs2 - 1) < 2.0 / n


def test_zero_pivot_sets_info():
    n = 40
    A = G.normal_matrix(n, 4)
    A[:, 13] = 0.0
    f = O.getrf(A, 8, 2)
    assert f.info == 14
    assert np.all(np.isfinite(f.LU))


def test_singular_zero_matrix():
    f = O.getrf(np.zeros((9, 9)), 4, 2)
    assert f.info == 1
    assert np.array_equal(f.ipiv, np.arange(9))


def test_prefix_panels_match_full_run():
    n, v = 300, 32
    A = G.normal_matrix(n, 9)
    full = O.getrf(A, v, 4)
    part = O.getrf(A, v, 4, npanels=3)
    k = 3 * v
    assert np.array_equal(part.ipiv[:k], full.ipiv[:k])
    assert np.array_equal(part.LU[:k, :], full.LU[:k, :])
    # Later panels interchange whole rows, L columns included: replay them.
    Lcols = part.LU[:, :k].copy()
    for i in range(k, n):
        r = full.ipiv[i]
        Lcols[[i, r]] = Lcols[[r, i]]
    assert np.array_equal(Lcols, full.LU[:, :k])


def test_thread_count_does_not_change_bits():
    code = (
        "import sys; sys.path.insert(0, %r);"
        "import numpy as np, cfx_inputs as G; from oracle import oracle as O;"
        "f = O.getrf(G.normal_matrix(400, 7), 32, 4);"
        "sys.stdout.write(f.LU.tobytes().hex()[:0] + str(hash(f.LU.tobytes())))" % ROOT)
    outs = []
    for t in ("1", "5"):
        env = dict(os.environ, OMP_NUM_THREADS=t, PYTHONHASHSEED="0")
        outs.append(subprocess.check_output([sys.executable, "-c", code], env=env))
    assert outs[0] == outs[1]


def test_argument_errors():
    with pytest.raises(ValueError):
        O.getrf(np.zeros((4, 4)), 0, 1)
    with pytest.raises(ValueError):
        O.getrf(np.zeros((4, 4)), 2, 0)
    with pytest.raises(ValueError):
        O.tslu(np.zeros((4, 4)), 5, 1)


# ---------------------------------------------------------------------------
# Solve and backward error
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,nrhs", [(64, 1), (200, 5), (257, 3)])
def test_getrs_matches_lapack_solve(n, nrhs):
    A = G.normal_matrix(n, 21)
    B = G.rhs(n, nrhs, 22)
    f = O.getrf(A, 16, 3)
    X = O.getrs(f.LU, f.ipiv, B)
    ref = sl.solve(A, B)
    np.testing.assert_allclose(X, ref, rtol=1e-9, atol=1e-9)
    assert O.eta(A, X, B) <= 1e-15


@pytest.mark.parametrize("cond", [1e2, 1e6])
def test_getrs_householder_closed_form(cond):
    n = 256
    spec = G.householder_spec(n, cond, 3)
    A = G.householder_matrix(spec)
    b = G.rhs(n, 1, 4)
    xs = G.householder_solution(spec, b)
    f = O.getrf(A, 32, 4)
    x = O.getrs(f.LU, f.ipiv, b)
    fe = np.abs(x - xs).max() / np.abs(xs).max()
    assert fe <= 50 * cond * 2.2e-16


def test_eta_exact_rational():
    rng = np.random.default_rng(0)
    n = 12
    A = rng.integers(-9, 10, size=(n, n)).astype(np.float64)
    x = rng.standard_normal(n)
    b = rng.standard_normal(n)
    Af = [[Fraction(int(a)) for a in r] for r in A]
    xf = [Fraction(float(t)) for t in x]
    bf = [Fraction(float(t)) for t in b]
    r = [bf[i] - sum(Af[i][j] * xf[j] for j in range(n)) for i in range(n)]
    num = max(abs(t) for t in r)
    den = max(sum(abs(a) for a in row) for row in Af) * max(abs(t) for t in xf) + max(abs(t) for t in bf)
    exact = float(num / den)
    assert O.eta(A, x, b) == pytest.approx(exact, rel=1e-14)


def test_eta_zero_for_exact_solution():
    rng = np.random.default_rng(1)
    A = rng.integers(-5, 6, size=(30, 30)).astype(np.float64)
    x = rng.integers(-5, 6, size=30).astype(np.float64)
    b = A @ x
    assert O.eta(A, x, b) == 0.0


def test_eta_catches_cancellation():
    """A residual that plain summation gets wrong: the exact residual is 1e-16
    relative to terms of size 1, which Dot2 resolves."""
    A = np.array([[1.0, 1e16, -1e16]])
    A = np.vstack([A, np.eye(3)[1:]])
    x = np.array([1.0, 1.0, 1.0])
    b = np.array([1.0, 1.0, 1.0])
    # r0 = 1 - (1 + 1e16 - 1e16) = 0 exactly; naive left-to-right gives 1.
    assert O.eta(A, x, b) == 0.0


def test_eta_compensation_recovers_lost_residual():
    """The opposite case: the exact residual is nonzero but plain summation
    loses it.  Row 0 gives r0 = 0 - (1e16 + 1 - 1e16) = -1 exactly, while
    left-to-right summation from b0 = 0 rounds -1e16 - 1 back to -1e16 (the
    spacing of doubles there is 2) and returns r0 = 0.  Exact eta =
    1 / (||A||_inf ||x||_inf + ||b||_inf) = 1 / (2e16 + 1 + 1)."""
    A = np.array([[1e16, 1.0, -1e16], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    x = np.ones(3)
    b = np.array([0.0, 1.0, 1.0])
    exact = float(Fraction(1) / (Fraction(2 * 10**16 + 1) + 1))
    assert O.eta(A, x, b) == pytest.approx(exact, rel=1e-15)
    assert O.eta(A, x, b) > 0.0


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
@pytest.mark.parametrize("where", ["x_one", "x_all", "b_one"])
def test_eta_non_finite_is_never_accurate(bad, where):
    """A non-finite solution (or right-hand side) must not score as a small
    backward error: eta is then NaN, so every "eta <= tol" check fails."""
    rng = np.random.default_rng(3)
    n = 16
    A = rng.standard_normal((n, n))
    x = rng.standard_normal(n)
    b = A @ x
    if where == "x_one":
        x[5] = bad
    elif where == "x_all":
        x[:] = bad
    else:
        b[7] = bad
    e = O.eta(A, x, b)
    assert not np.isfinite(e)
    assert not (e <= 5e-15)


def test_eta_non_finite_matrix_entry():
    """An infinite entry of A met by the residual makes eta NaN as well."""
    A = np.eye(4)
    A[2, 1] = np.inf
    x = np.ones(4)
    b = np.ones(4)
    assert not np.isfinite(O.eta(A, x, b))


def test_eta_max_over_columns_keeps_nan():
    """Several right-hand sides: a NaN column is not hidden by a later finite one."""
    A = np.eye(3)
    X = np.ones((3, 2))
    B = np.ones((3, 2))
    X[0, 0] = np.nan
    assert not np.isfinite(O.eta(A, X, B))


# ---------------------------------------------------------------------------
# Generators with closed forms
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("cond", [1e2, 1e6, 1e10])
def test_householder_generator_condition(cond):
    n = 64
    spec = G.householder_spec(n, cond, 5)
    A = G.householder_matrix(spec)
    s = np.linalg.svd(A, compute_uv=False)
    np.testing.assert_allclose(s, spec.s, rtol=1e-10 * max(1.0, cond / 1e6))
    sign, logdet = np.linalg.slogdet(A)
    assert sign == 1.0
    assert logdet == pytest.approx(np.log(spec.s).sum(), rel=1e-8, abs=1e-8)


# ---------------------------------------------------------------------------
# Minimum leaf height: the leaf count follows the panel's height
# ---------------------------------------------------------------------------

def test_min_leaf_rows_extremes():
    """R >= n gives one leaf per panel: TP(v, 1), i.e. the same factors as
    L = 1; R = 1 gives min(L, rows) = L leaves: the fixed-L factors."""
    A = G.normal_matrix(200, 71)
    one = O.getrf(A, 16, 1)
    r_big = O.getrf(A, 16, 8, min_leaf_rows=500)
    assert np.array_equal(r_big.ipiv, one.ipiv) and np.array_equal(r_big.LU, one.LU)
    fixed = O.getrf(A, 16, 8)
    r_one = O.getrf(A, 16, 8, min_leaf_rows=1)
    assert np.array_equal(r_one.ipiv, fixed.ipiv) and np.array_equal(r_one.LU, fixed.LU)
    with pytest.raises(ValueError):
        O.getrf(A, 16, 8, min_leaf_rows=-1)


def test_min_leaf_rows_per_panel_leaf_count():
    """n = 480, v = 32, L = 4, R = 128: panel j (r = 480 - 32 j rows) has
    min(4, ceil(r / 128)) leaves -- 4, 4, 4, 3, 3, 3, 3, 2, 2, 2, 2, 1, ...
    Each panel step of the full factorisation equals one panel of a
    fixed-leaf factorisation of the trailing matrix left by the previous
    panels, with that leaf count (pivots and values bit for bit)."""
    n, v, L, R = 480, 32, 4, 128
    expect = [4, 4, 4, 3, 3, 3, 3, 2, 2, 2, 2, 1, 1, 1, 1]
    A = G.normal_matrix(n, 72)
    for j, lj in enumerate(expect):
        k = j * v
        before = O.getrf(A, v, L, npanels=j, min_leaf_rows=R) if j else None
        T = (before.LU if j else A)[k:, k:].copy()
        step = O.getrf(T, v, lj, npanels=1)
        full = O.getrf(A, v, L, npanels=j + 1, min_leaf_rows=R)
        assert np.array_equal(full.ipiv[k:k + v] - k, step.ipiv[:v]), j
        assert np.array_equal(full.LU[k:, k:], step.LU), j
        # a different leaf count gives different pivots on this matrix for
        # the panels where the rule decides (the pin would catch a wrong count)
        if lj > 1:
            other = O.getrf(T, v, lj - 1, npanels=1)
            assert not np.array_equal(other.ipiv[:v], step.ipiv[:v]) or not np.array_equal(other.LU, step.LU)
