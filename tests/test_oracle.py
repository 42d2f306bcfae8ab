"""Pins of the CPU oracle against facts fixed by the mathematics (no GPU).

Each pin checks the oracle against something other than itself:
brute-force dense factorization/inversion, the exactly known factor of the
synthetic inputs, exact rational arithmetic, LAPACK special cases, block
identities of Sigma*Q, closed-form log-determinants and torch autograd.  The
mutation tests at the end plant plausible mistakes in the oracle and check that
one of the pins catches each of them.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.linalg import lapack

import oracle
from oracle import bta_oracle as ob
from paper_2503_17528_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TINY = [(1, 3, 0), (1, 4, 2), (2, 3, 1), (2, 1, 1), (3, 5, 0), (4, 5, 3), (5, 2, 4), (3, 16, 3)]


def _random_spd_bta(n, b, a, seed):
    """A random SPD BTA matrix that does not come from the LL^T generator:
    random blocks, then a diagonal shift that makes it diagonally dominant."""
    rng = np.random.default_rng(seed)
    D = rng.standard_normal((n, b, b))
    D = 0.5 * (D + np.transpose(D, (0, 2, 1)))
    B = rng.standard_normal((max(n - 1, 0), b, b))
    R = rng.standard_normal((n, a, b))
    T = rng.standard_normal((a, a))
    T = 0.5 * (T + T.T)
    Q = _dense_independent(D, B, R, T)
    shift = np.max(np.sum(np.abs(Q), axis=1)) + 1.0
    for i in range(n):
        D[i] += shift * np.eye(b)
    T += shift * np.eye(a)
    # put garbage in the strict upper triangles: only lower triangles are read
    for i in range(n):
        D[i] += np.triu(rng.standard_normal((b, b)) * 100.0, 1)
    if a:
        T += np.triu(rng.standard_normal((a, a)) * 100.0, 1)
    return D, B, R, T


def _blocks(F):
    return {"D": F["LD"], "B": F["LB"], "R": F["LR"], "T": F["LT"]}


def _xblocks(X):
    return {"D": X["XD"], "B": X["XB"], "R": X["XR"], "T": X["XT"]}


# ---------------------------------------------------------------------------
# brute force against dense LAPACK at tiny sizes


@pytest.mark.parametrize("n,b,a", TINY)
@pytest.mark.parametrize("seed", [0, 1])
def test_factor_matches_dense_cholesky(n, b, a, seed):
    D, B, R, T = _random_spd_bta(n, b, a, seed)
    F = oracle.pobtaf(D, B, R, T)
    assert F["info"] == 0
    Ld = np.linalg.cholesky(oracle.dense(D, B, R, T))
    e = oracle.rel_block_errors(_blocks(F), oracle.pattern(Ld, n, b, a))
    assert max(e.values()) < 1e-13, e
    # fill-in stays inside the pattern: everything else of the dense factor is zero
    mask = np.abs(oracle.dense_lower_factor(F["LD"], F["LB"], F["LR"], F["LT"])) > 0
    assert np.all(np.abs(Ld[~mask]) < 1e-12)
    # exact zeros above the diagonal of the diagonal blocks and the tip
    for i in range(n):
        assert np.all(np.triu(F["LD"][i], 1) == 0.0)
    assert np.all(np.triu(F["LT"], 1) == 0.0)


@pytest.mark.parametrize("n,b,a", TINY)
@pytest.mark.parametrize("seed", [0, 1])
def test_selinv_matches_dense_inverse(n, b, a, seed):
    D, B, R, T = _random_spd_bta(n, b, a, seed)
    F = oracle.pobtaf(D, B, R, T)
    X = oracle.pobtasi(F["LD"], F["LB"], F["LR"], F["LT"])
    S = np.linalg.inv(oracle.dense(D, B, R, T))
    e = oracle.rel_block_errors(_xblocks(X), oracle.pattern(S, n, b, a), lower_keys=())
    assert max(e.values()) < 1e-12, e
    # returned symmetric blocks are exactly symmetric
    for i in range(n):
        assert np.array_equal(X["XD"][i], X["XD"][i].T)
    assert np.array_equal(X["XT"], X["XT"].T)


@pytest.mark.parametrize("n,b,a", TINY)
def test_solve_and_logdet_match_dense(n, b, a):
    D, B, R, T = _random_spd_bta(n, b, a, 7)
    F = oracle.pobtaf(D, B, R, T)
    Q = oracle.dense(D, B, R, T)
    y = np.random.default_rng(3).standard_normal((n * b + a, 3))
    x = oracle.pobtas(F["LD"], F["LB"], F["LR"], F["LT"], y)
    assert np.max(np.abs(x - np.linalg.solve(Q, y))) / np.max(np.abs(x)) < 1e-12
    x1 = oracle.pobtas(F["LD"], F["LB"], F["LR"], F["LT"], y[:, 0])
    assert x1.shape == (n * b + a,)
    assert np.allclose(x1, x[:, 0], rtol=0, atol=1e-14 * np.max(np.abs(x)))
    sign, ld = np.linalg.slogdet(Q)
    assert sign == 1.0
    assert abs(oracle.logdet(F["LD"], F["LT"]) - ld) < 1e-11 * max(1.0, abs(ld))


# ---------------------------------------------------------------------------
# exact rational example (tests/golden)


def test_exact_rational_example():
    with open(os.path.join(GOLDEN, "exact_bta_n3_b2_a1.json")) as f:
        g = json.load(f)
    n, b, a = g["n"], g["b"], g["a"]
    fl = lambda M: np.array([[float(Fraction(v)) for v in r] for r in M])
    Q, L, S = fl(g["Q"]), fl(g["L"]), fl(g["Sigma"])
    blocks = oracle.pattern(Q, n, b, a)
    F = oracle.pobtaf(blocks["D"], blocks["B"], blocks["R"], blocks["T"])
    assert F["info"] == 0
    e = oracle.rel_block_errors(_blocks(F), oracle.pattern(L, n, b, a))
    assert max(e.values()) < 1e-15, e
    X = oracle.pobtasi(F["LD"], F["LB"], F["LR"], F["LT"])
    e = oracle.rel_block_errors(_xblocks(X), oracle.pattern(S, n, b, a), lower_keys=())
    assert max(e.values()) < 1e-14, e
    y = np.array([float(Fraction(v)) for v in g["y"]])
    x = np.array([float(Fraction(v)) for v in g["x"]])
    assert np.max(np.abs(oracle.pobtas(F["LD"], F["LB"], F["LR"], F["LT"], y) - x)) < 1e-13 * np.max(np.abs(x))
    assert abs(oracle.logdet(F["LD"], F["LT"]) - math.log(float(Fraction(g["det_Q"])))) < 1e-13


# ---------------------------------------------------------------------------
# known factor of the synthetic inputs


@pytest.mark.parametrize("wl", [synth.SMALL, synth.workload(6, 40, 3), synth.workload(3, 96, 0),
                                synth.workload(4, 128, 6, "scaled", diag=(1, 3)),
                                synth.workload(4, 32, 128, "scaled")], ids=lambda w: w.name)
def test_recovers_known_factor(wl):
    Q = synth.make_np(wl, 11, with_factor=True)
    F = oracle.pobtaf(Q["D"], Q["B"], Q["R"], Q["T"])
    assert F["info"] == 0
    e = oracle.rel_block_errors(_blocks(F), {"D": Q["LD"], "B": Q["LB"], "R": Q["LR"], "T": Q["LT"]})
    assert max(e.values()) < 1e-12, e
    # closed-form log-determinant from the drawn factor
    ld = 2.0 * (np.sum(np.log(np.diagonal(Q["LD"], axis1=1, axis2=2))) + np.sum(np.log(np.diag(Q["LT"]))))
    assert abs(oracle.logdet(F["LD"], F["LT"]) - ld) < 1e-12 * abs(ld)


@pytest.mark.parametrize("wl", [synth.SMALL, synth.workload(5, 64, 0), synth.workload(8, 48, 5),
                                synth.workload(4, 32, 128, "scaled")], ids=lambda w: w.name)
def test_sigma_times_q_pattern_identities(wl):
    """(Sigma Q)_jj = I, (Sigma Q)_{n,j} = 0, (Sigma Q)_nn = I use only selected
    blocks of Sigma, so they check X at any size."""
    Q = synth.make_np(wl, 5)
    n, b, a = wl.n, wl.b, wl.a
    F = oracle.pobtaf(Q["D"], Q["B"], Q["R"], Q["T"])
    X = oracle.pobtasi(F["LD"], F["LB"], F["LR"], F["LT"])
    D, B, R, T = Q["D"], Q["B"], Q["R"], Q["T"]
    XD, XB, XR, XT = X["XD"], X["XB"], X["XR"], X["XT"]
    tol = 1e-12
    for j in range(n):
        # row block j of Sigma times column block j of Q
        acc = XD[j] @ D[j] + XR[j].T @ R[j]
        if j > 0:
            acc += XB[j - 1] @ B[j - 1].T
        if j < n - 1:
            acc += XB[j].T @ B[j]
        assert np.max(np.abs(acc - np.eye(b))) < tol
        # row block n of Sigma times column block j of Q
        acc = XR[j] @ D[j] + XT @ R[j]
        if j > 0:
            acc += XR[j - 1] @ B[j - 1].T
        if j < n - 1:
            acc += XR[j + 1] @ B[j]
        if a:
            assert np.max(np.abs(acc)) < tol
    if a:
        acc = XT @ T + sum(XR[j] @ R[j].T for j in range(n))
        assert np.max(np.abs(acc - np.eye(a))) < tol


def test_sampled_columns_of_sigma():
    """Sigma e_c = Q^{-1} e_c via a dense solve, compared with the selected
    entries of that column."""
    wl = synth.workload(6, 24, 3)
    Q = synth.make_np(wl, 2)
    n, b, a = wl.n, wl.b, wl.a
    Qd = oracle.dense(Q["D"], Q["B"], Q["R"], Q["T"])
    F = oracle.pobtaf(Q["D"], Q["B"], Q["R"], Q["T"])
    X = oracle.pobtasi(F["LD"], F["LB"], F["LR"], F["LT"])
    rng = np.random.default_rng(0)
    for c in rng.choice(wl.N, 12, replace=False):
        col = np.linalg.solve(Qd, np.eye(wl.N)[:, c])
        if c < n * b:
            j, cc = divmod(int(c), b)
            assert np.allclose(X["XD"][j][:, cc], col[j * b:(j + 1) * b], atol=1e-13)
            if j < n - 1:
                assert np.allclose(X["XB"][j][:, cc], col[(j + 1) * b:(j + 2) * b], atol=1e-13)
            assert np.allclose(X["XR"][j][:, cc], col[n * b:], atol=1e-13)
        else:
            cc = int(c) - n * b
            assert np.allclose(X["XT"][:, cc], col[n * b:], atol=1e-13)
            for j in range(n):
                assert np.allclose(X["XR"][j][cc, :], col[j * b:(j + 1) * b], atol=1e-13)


# ---------------------------------------------------------------------------
# special cases that reduce to textbook routines


@pytest.mark.parametrize("b,a", [(7, 0), (7, 3), (33, 5)])
def test_single_block_is_dense_potrf_potri(b, a):
    """n = 1: the BTA matrix is one dense (b+a) x (b+a) SPD matrix."""
    D, B, R, T = _random_spd_bta(1, b, a, 4)
    Q = oracle.dense(D, B, R, T)
    c, info = lapack.dpotrf(Q, lower=1, clean=1)
    assert info == 0
    F = oracle.pobtaf(D, B, R, T)
    e = oracle.rel_block_errors(_blocks(F), oracle.pattern(np.tril(c), 1, b, a))
    assert max(e.values()) < 1e-14
    inv, info = lapack.dpotri(c, lower=1)
    assert info == 0
    inv = np.tril(inv) + np.tril(inv, -1).T
    X = oracle.pobtasi(F["LD"], F["LB"], F["LR"], F["LT"])
    e = oracle.rel_block_errors(_xblocks(X), oracle.pattern(inv, 1, b, a), keys=("D", "R", "T"), lower_keys=())
    assert max(e.values()) < 1e-12


def test_block_diagonal_special_case():
    """B = R = 0: every selected diagonal block is the inverse of its own block."""
    n, b, a = 4, 9, 3
    D, B, R, T = _random_spd_bta(n, b, a, 9)
    B[:] = 0
    R[:] = 0
    F = oracle.pobtaf(D, B, R, T)
    X = oracle.pobtasi(F["LD"], F["LB"], F["LR"], F["LT"])
    for i in range(n):
        Di = np.tril(D[i]) + np.tril(D[i], -1).T
        assert np.allclose(X["XD"][i], np.linalg.inv(Di), rtol=1e-12, atol=1e-14)
        assert np.all(X["XR"][i] == 0)
    assert np.all(X["XB"] == 0)
    Tm = np.tril(T) + np.tril(T, -1).T
    assert np.allclose(X["XT"], np.linalg.inv(Tm), rtol=1e-12, atol=1e-14)


def test_block_tridiagonal_a0_equals_dense_banded():
    """a = 0 is the BT case: compare with scipy's banded Cholesky solver."""
    n, b = 5, 4
    D, B, R, T = _random_spd_bta(n, b, 0, 12)
    Q = oracle.dense(D, B, R, T)
    N = n * b
    bw = 2 * b - 1
    ab = np.zeros((bw + 1, N))
    for j in range(N):
        for i in range(j, min(N, j + bw + 1)):
            ab[i - j, j] = Q[i, j]
    cb = sla.cholesky_banded(ab, lower=True)
    F = oracle.pobtaf(D, B, R, T)
    Ld = oracle.dense_lower_factor(F["LD"], F["LB"], F["LR"], F["LT"])
    for j in range(N):
        for i in range(j, min(N, j + bw + 1)):
            assert abs(Ld[i, j] - cb[i - j, j]) < 1e-13 * max(1.0, abs(cb[i - j, j]))


# ---------------------------------------------------------------------------
# failure reporting


@pytest.mark.parametrize("where", ["first", "middle", "last", "tip"])
@pytest.mark.parametrize("bad", [-1.0, np.nan])
def test_failure_reports_global_row(where, bad):
    n, b, a = 4, 6, 3
    D, B, R, T = _random_spd_bta(n, b, a, 21)
    if where == "tip":
        T[1, 1] = bad if np.isnan(bad) else -1e6
        expect = n * b + 2
    else:
        blk = {"first": 0, "middle": 2, "last": n - 1}[where]
        D[blk][3, 3] = bad if np.isnan(bad) else -1e6
        expect = blk * b + 4
    F = oracle.pobtaf(D, B, R, T)
    assert F["info"] == expect


# ---------------------------------------------------------------------------
# gradient of f(Q) = logdet Q + y^T Q^{-1} y


def _grad_case(n, b, a, seed):
    D, B, R, T = _random_spd_bta(n, b, a, seed)
    # symmetric inputs for the autograd convention
    for i in range(n):
        D[i] = np.tril(D[i]) + np.tril(D[i], -1).T
    T = np.tril(T) + np.tril(T, -1).T
    y = np.random.default_rng(seed + 1).standard_normal(n * b + a)
    return D, B, R, T, y


def _oracle_grad(D, B, R, T, y):
    n, b, a = D.shape[0], D.shape[1], T.shape[0]
    F = oracle.pobtaf(D, B, R, T)
    X = oracle.pobtasi(F["LD"], F["LB"], F["LR"], F["LT"])
    x = oracle.pobtas(F["LD"], F["LB"], F["LR"], F["LT"], y)
    f = oracle.logdet(F["LD"], F["LT"]) + float(y @ x)
    return f, oracle.grad_logdet_quad(X, x, n, b, a)


@pytest.mark.parametrize("n,b,a", [(3, 4, 2), (2, 5, 0), (4, 3, 3)])
def test_gradient_matches_torch_autograd_dense(n, b, a):
    torch = pytest.importorskip("torch")
    D, B, R, T, y = _grad_case(n, b, a, 30)
    f, G = _oracle_grad(D, B, R, T, y)
    tD, tB, tR, tT = (torch.tensor(v, dtype=torch.float64, requires_grad=True) for v in (D, B, R, T))
    N = n * b + a
    Q = torch.zeros((N, N), dtype=torch.float64)
    Q = Q.clone()
    rows = []
    # assemble with index_put so autograd sees every use
    for i in range(n):
        s = slice(i * b, (i + 1) * b)
        Q[s, s] = 0.5 * (tD[i] + tD[i].T)
        if i < n - 1:
            s1 = slice((i + 1) * b, (i + 2) * b)
            Q[s1, s] = tB[i]
            Q[s, s1] = tB[i].T
        Q[n * b:, s] = tR[i]
        Q[s, n * b:] = tR[i].T
    Q[n * b:, n * b:] = 0.5 * (tT + tT.T)
    ty = torch.tensor(y, dtype=torch.float64)
    fv = torch.logdet(Q) + ty @ torch.linalg.solve(Q, ty)
    fv.backward()
    assert abs(fv.item() - f) < 1e-11 * abs(f)
    for k, t in (("D", tD), ("B", tB), ("R", tR), ("T", tT)):
        ref = t.grad.numpy()
        if ref.size:
            assert np.max(np.abs(G[k] - ref)) < 1e-11 * max(1.0, np.max(np.abs(ref))), k


def test_gradient_directional_finite_difference():
    n, b, a = 4, 6, 2
    D, B, R, T, y = _grad_case(n, b, a, 40)
    f0, G = _oracle_grad(D, B, R, T, y)
    rng = np.random.default_rng(41)
    V = {k: rng.standard_normal(v.shape) for k, v in (("D", D), ("B", B), ("R", R), ("T", T))}
    V["D"] = 0.5 * (V["D"] + np.transpose(V["D"], (0, 2, 1)))
    V["T"] = 0.5 * (V["T"] + V["T"].T)
    h = 1e-6
    fp, _ = _oracle_grad(D + h * V["D"], B + h * V["B"], R + h * V["R"], T + h * V["T"], y)
    fm, _ = _oracle_grad(D - h * V["D"], B - h * V["B"], R - h * V["R"], T - h * V["T"], y)
    fd = (fp - fm) / (2 * h)
    inner = sum(float(np.sum(G[k] * V[k])) for k in V)
    assert abs(fd - inner) < 1e-6 * max(1.0, abs(inner))


def test_gradient_at_zero_rhs_is_selected_inverse():
    n, b, a = 3, 5, 2
    D, B, R, T, _ = _grad_case(n, b, a, 50)
    _, G = _oracle_grad(D, B, R, T, np.zeros(n * b + a))
    S = np.linalg.inv(oracle.dense(D, B, R, T))
    P = oracle.pattern(S, n, b, a)
    assert np.allclose(G["D"], P["D"], atol=1e-13)
    assert np.allclose(G["B"], 2 * P["B"], atol=1e-13)
    assert np.allclose(G["R"], 2 * P["R"], atol=1e-13)
    assert np.allclose(G["T"], P["T"], atol=1e-13)


# ---------------------------------------------------------------------------
# mutation tests: a planted mistake in the oracle must fail a pin


def _dense_independent(D, B, R, T):
    """Dense assembly written out with np.block, independent of the oracle."""
    n, b, a = D.shape[0], D.shape[1], T.shape[0]
    Z = lambda r, c: np.zeros((r, c))
    sym = lambda M: np.tril(M) + np.tril(M, -1).T
    rows = []
    for i in range(n):
        row = []
        for j in range(n):
            if i == j:
                row.append(sym(D[i]))
            elif i == j + 1:
                row.append(B[j])
            elif j == i + 1:
                row.append(B[i].T)
            else:
                row.append(Z(b, b))
        row.append(R[i].T)
        rows.append(row)
    rows.append([R[j] for j in range(n)] + [sym(T)])
    return np.block(rows)


def _pins_pass():
    """The brute-force pins at two tiny sizes (with and without an arrow).
    An exception raised by a mutated oracle counts as a caught mistake."""
    try:
        return _pins_pass_inner()
    except Exception:
        return False


def _pins_pass_inner():
    ok = True
    for (n, b, a) in [(4, 5, 3), (3, 4, 0)]:
        D, B, R, T = _random_spd_bta(n, b, a, 1)
        Qd = _dense_independent(D, B, R, T)
        F = oracle.pobtaf(D, B, R, T)
        eL = oracle.rel_block_errors(_blocks(F), oracle.pattern(np.linalg.cholesky(Qd), n, b, a))
        X = oracle.pobtasi(F["LD"], F["LB"], F["LR"], F["LT"])
        eX = oracle.rel_block_errors(_xblocks(X), oracle.pattern(np.linalg.inv(Qd), n, b, a), lower_keys=())
        y = np.arange(n * b + a, dtype=float) - 2.0
        x = oracle.pobtas(F["LD"], F["LB"], F["LR"], F["LT"], y)
        ok &= max(eL.values()) < 1e-12 and max(eX.values()) < 1e-12
        ok &= np.allclose(Qd @ x, y, atol=1e-10)
        ok &= abs(oracle.logdet(F["LD"], F["LT"]) - np.linalg.slogdet(Qd)[1]) < 1e-10
    return ok


def test_pins_pass_on_the_real_oracle():
    assert _pins_pass()


MUTATIONS = {
    # Algorithm 1 solve uses L^{-1} instead of L^{-T}
    "trsm_no_transpose": ("_trsm_right_lower_trans", lambda L, Bm: ob._trsm_right_lower(L, Bm)),
    # Algorithm 2 solve uses L^{-T} instead of L^{-1}
    "selinv_trsm_transposed": ("_trsm_right_lower", lambda L, U: ob._trsm_right_lower_trans.__wrapped__(L, U)
                               if hasattr(ob._trsm_right_lower_trans, "__wrapped__") else
                               (np.zeros_like(U) if U.size == 0 else sla.solve_triangular(L, U.T, lower=True, trans="N").T)),
    # inverse of L returned transposed
    "inv_transposed": ("_inv_lower", lambda L: (np.zeros((0, 0)) if L.shape[0] == 0 else
                                                sla.solve_triangular(L, np.eye(L.shape[0]), lower=True).T)),
    # factorization reads the upper triangle of the diagonal blocks
    "potrf_reads_upper": ("_potrf", lambda A: (np.tril(lapack.dpotrf(np.array(A.T, order="F"), lower=1, clean=1)[0]),
                                               int(lapack.dpotrf(np.array(A.T, order="F"), lower=1, clean=1)[1]))),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(monkeypatch, name):
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(ob, attr, fn)
    assert not _pins_pass(), f"planted mistake {name} was not caught"


def test_planted_dropped_term_is_caught(monkeypatch):
    """Dropping the arrow update of the tip (A_nn -= L_{n,i} L_{n,i}^T) or
    the sign of a U term must fail the brute-force pins."""
    real_pobtasi = ob.pobtasi

    def wrong_sign(LD, LB, LR, LT):
        X = real_pobtasi(LD, LB, LR, LT)
        X["XB"] = -X["XB"]
        return X

    monkeypatch.setattr(oracle, "pobtasi", wrong_sign)
    assert not _pins_pass()
    monkeypatch.setattr(oracle, "pobtasi", real_pobtasi)

    real_pobtaf = ob.pobtaf

    def no_tip_update(D, B, R, T):
        F = real_pobtaf(D, B, R, T)
        # recompute the tip factor without the arrow contributions
        F["LT"], _ = ob._potrf(np.asarray(T))
        return F

    monkeypatch.setattr(oracle, "pobtaf", no_tip_update)
    assert not _pins_pass()
