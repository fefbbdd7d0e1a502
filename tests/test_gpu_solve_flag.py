"""Error reporting of the one-launch triangular solves, and the ordering of
getrs calls that share a handle.

The give-up path is forced from the host: a spin limit of 0 polls makes every
block that would have to wait give up at once, so every kernel still exits
normally (no wait is ever unbounded).  Every call goes through the C ABI."""
import numpy as np
import pytest

import cfx_inputs as G
from oracle import oracle as O
from tests.gpu_util import say, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ESOLVE = -1005


@pytest.fixture(scope="module")
def cfx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2010_05975_amd import cfx as m
    m.lib()
    return m


def factor(cfx, n, seed, handle=None):
    A = G.normal_matrix(n, seed)
    dA = to_dev(A)
    ipiv, info = cfx.getrf(dA, v=64, leaves=4, handle=handle)
    torch.cuda.synchronize()
    assert int(info.cpu()[0]) == 0
    return A, dA, ipiv


def test_getrs_check_clean(cfx):
    say("getrs check after a normal one-RHS solve")
    A, dA, ipiv = factor(cfx, 3000, 71)
    b = G.rhs(3000, 1, 72)
    db = to_dev(b)
    cfx.getrs(dA, ipiv, db)
    assert cfx.getrs_check() == 0
    assert O.eta(A, db.cpu().numpy(), b) <= 5e-15


def test_forced_give_up_is_reported(cfx):
    n = 8192
    say(f"forced give-up of the one-RHS solve, n={n}")
    h = cfx.Handle()
    try:
        A, dA, ipiv = factor(cfx, n, 73, handle=h)
        b = G.rhs(n, 1, 74)
        cfx.set_solve_spin_limit(0, handle=h)
        db = to_dev(b)
        cfx.getrs(dA, ipiv, db, handle=h)
        assert cfx.getrs_check(handle=h) == ESOLVE
        x = db.cpu().numpy()
        assert np.isnan(x).any(), "a block that gave up must leave NaN"
        assert not (O.eta(A, x, b) <= 5e-15)
        # the flag was cleared by the check; the default limit solves again
        cfx.set_solve_spin_limit(1 << 22, handle=h)
        db = to_dev(b)
        cfx.getrs(dA, ipiv, db, handle=h)
        assert cfx.getrs_check(handle=h) == 0
        assert O.eta(A, db.cpu().numpy(), b) <= 5e-15
    finally:
        h.close()


def test_forced_give_up_in_refinement_is_an_error(cfx):
    n = 4096
    say(f"forced give-up inside gesv_ir, n={n}")
    h = cfx.Handle()
    try:
        A = G.normal_matrix(n, 75)
        b = G.rhs(n, 1, 76)
        dA, db = to_dev(A), to_dev(b)
        cfx.set_solve_spin_limit(0, handle=h)
        with pytest.raises(cfx.CfxError) as e:
            cfx.gesv_ir(dA, db, handle=h, precision="fp64", v=64, leaves=4, max_outer=2)
        assert e.value.code == ESOLVE
        cfx.set_solve_spin_limit(1 << 22, handle=h)
        x, rep = cfx.gesv_ir(dA, db, handle=h, precision="fp64", v=64, leaves=4, max_outer=2)
        assert rep["converged"] == 1
        assert O.eta(A, x.cpu().numpy(), b) <= 5e-15
    finally:
        h.close()


def test_getrs_on_two_streams_share_the_handle_safely(cfx):
    """Two getrs calls on one handle, issued on different streams without any
    ordering by the caller: the handle orders them, so both results equal the
    results of the same calls on one stream, bit for bit."""
    n = 4000
    say(f"getrs on two streams, one handle, n={n}")
    A, dA, ipiv = factor(cfx, n, 77)
    b1, b2 = G.rhs(n, 1, 78), G.rhs(n, 3, 79)
    want = []
    for b in (b1, b2):
        db = to_dev(b)
        cfx.getrs(dA, ipiv, db)
        torch.cuda.synchronize()
        want.append(db.cpu().numpy())
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    d1, d2 = to_dev(b1), to_dev(b2)
    torch.cuda.synchronize()
    for rep in range(3):
        d1.copy_(to_dev(b1))
        d2.copy_(to_dev(b2))
        torch.cuda.synchronize()
        cfx.getrs(dA, ipiv, d1, stream=s1)
        cfx.getrs(dA, ipiv, d2, stream=s2)
        torch.cuda.synchronize()
        assert np.array_equal(d1.cpu().numpy(), want[0]), rep
        assert np.array_equal(d2.cpu().numpy(), want[1]), rep
    assert cfx.getrs_check() == 0
