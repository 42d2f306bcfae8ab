"""Writes ``exact_bta_n3_b2_a1.json``: a tiny BTA matrix whose Cholesky factor,
selected inverse, log-determinant and solve are known exactly.

The factor L is chosen with power-of-two diagonal entries and small integer
off-diagonal entries, so L^{-1}, Sigma = L^{-T} L^{-1} and x = Sigma y are
dyadic rationals, exactly representable in binary floating point.  Everything
is computed with Python's exact ``fractions`` arithmetic from the definitions
(Q = L L^T, Sigma = Q^{-1}); neither the oracle nor the HIP path is used.
Run from the repository root: ``python tests/golden/make_golden.py``.
"""
import json
import os
from fractions import Fraction as F

n, b, a = 3, 2, 1
N = n * b + a
# block lower-triangular factor with the BTA pattern (rows/cols 0..6; tip = row 6)
L = [[F(0)] * N for _ in range(N)]
diag = [2, 1, 4, 2, 1, 2, 4]
for k in range(N):
    L[k][k] = F(diag[k])
L[1][0] = F(1)            # inside L_00
L[3][2] = F(-1)           # inside L_11
L[5][4] = F(3)            # inside L_22
L[2][0], L[2][1], L[3][0], L[3][1] = F(1), F(-2), F(0), F(1)      # L_10
L[4][2], L[4][3], L[5][2], L[5][3] = F(2), F(1), F(-1), F(1)      # L_21
L[6][0], L[6][1], L[6][2], L[6][3], L[6][4], L[6][5] = F(1), F(0), F(-1), F(2), F(1), F(-3)  # L_{n,i}


def matmul(X, Y):
    return [[sum(X[i][k] * Y[k][j] for k in range(len(Y))) for j in range(len(Y[0]))] for i in range(len(X))]


def transpose(X):
    return [list(r) for r in zip(*X)]


def inv_lower(Lm):
    m = len(Lm)
    W = [[F(0)] * m for _ in range(m)]
    for j in range(m):
        W[j][j] = 1 / Lm[j][j]
        for i in range(j + 1, m):
            W[i][j] = -sum(Lm[i][k] * W[k][j] for k in range(j, i)) / Lm[i][i]
    return W


Q = matmul(L, transpose(L))
W = inv_lower(L)
S = matmul(transpose(W), W)
y = [F(v) for v in (1, -1, 2, 0, 3, -2, 1)]
x = [sum(S[i][j] * y[j] for j in range(N)) for i in range(N)]
# check: Q S = I exactly
QS = matmul(Q, S)
assert all(QS[i][j] == (1 if i == j else 0) for i in range(N) for j in range(N))
# log det Q = 2 * sum log L_kk = 2 * log(prod diag) (prod is an integer here)
prod = 1
for d in diag:
    prod *= d

s = lambda M: [[str(v) for v in r] for r in M]
doc = {
    "description": "exact BTA example n=3 b=2 a=1; values are exact rationals as strings",
    "n": n, "b": b, "a": a,
    "Q": s(Q), "L": s(L), "Sigma": s(S), "y": [str(v) for v in y], "x": [str(v) for v in x],
    "det_Q": str(F(prod) ** 2),
}
here = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(here, "exact_bta_n3_b2_a1.json"), "w") as f:
    json.dump(doc, f, indent=1)
print("wrote", os.path.join(here, "exact_bta_n3_b2_a1.json"))
