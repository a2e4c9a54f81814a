"""CPU emulation of the literal scheme's per-anchor factorisation on its lane grids (CPU only).

k_lit_anchor (csrc/fbsde_literal.hip) spreads the bordered (M + 1) x (M + 1) anchor system over an RI x RJ
lane grid: lane (r, c) holds the entries (r + RI a, c + RJ b), b <= bmax(a) = (RI a + RI - 1) // RJ, a < A.
Elimination step jp (pivot column block JB = jp // RJ) has the lanes of column jp write their entries of
that column into one of two column buffers of CW = max(RI A, RJ B) doubles, then every lane updates its
entries right of the pivot; the back substitution has the lanes of row jp update the right-hand side.

This test replays that index logic lane by lane for every layout the library instantiates (and the 8 x 8
grid with 13 row blocks, which is not instantiated) and checks:
* every buffer index stays below CW and every right-hand-side index below M;
* every buffer entry a step reads was written in that step (a stale entry from two steps earlier would be
  a wrong value that no bound check sees);
* the solution equals a dense solve of the same system to rounding.
"""
import numpy as np
import pytest


def bmax(RI, RJ, a):
    return (RI * a + RI - 1) // RJ


def amin(RI, RJ, b):
    a = 0
    while bmax(RI, RJ, a) < b:
        a += 1
    return a


def emulate(RI, RJ, A, M, rng, specialised):
    n = M + 1
    B = bmax(RI, RJ, A - 1) + 1
    CW = max(RI * A, RJ * B)
    assert RI * A >= n and RJ * B >= n
    # a symmetric positive definite system with a bordered right-hand-side row
    X = rng.normal(size=(M, M + 3))
    K = X @ X.T / M + 0.5 * np.eye(M)
    y = rng.normal(size=M)
    S = np.zeros((RI * A, RJ * B))
    S[:M, :M] = np.tril(K)
    S[M, :M] = y
    # lane-resident slots: v[(r, c)][(a, b)]
    v = {}
    for r in range(RI):
        for c in range(RJ):
            for a in range(A):
                for b in range(bmax(RI, RJ, a) + 1):
                    i, j = r + RI * a, c + RJ * b
                    v[(r, c, a, b)] = S[i, j] if (i < n and j <= i) else 0.0
    col = [np.full(CW, np.nan), np.full(CW, np.nan)]
    stamp = [np.full(CW, -1), np.full(CW, -1)]
    for jp in range(M):
        cb, st = col[jp & 1], stamp[jp & 1]
        JB, jr = jp // RJ, jp % RJ
        a0 = amin(RI, RJ, JB) if specialised else 0
        for r in range(RI):
            for a in range(a0, A):
                if JB <= bmax(RI, RJ, a):
                    idx = r + RI * a
                    assert idx < CW
                    cb[idx] = v[(r, jr, a, JB)]
                    st[idx] = jp
        assert st[jp] == jp
        dj = cb[jp]
        new = {}
        for (r, c, a, b), x in v.items():
            if a < a0 or b < JB:
                continue
            if not (b > JB or c > jr):
                continue
            ri, ci = r + RI * a, c + RJ * b
            assert ri < CW and ci < CW
            # both operands must come from this step's writes
            assert st[ri] == jp and st[ci] == jp, (RI, RJ, A, M, jp, ri, ci)
            new[(r, c, a, b)] = x - cb[ri] * (cb[ci] / dj)
        v.update(new)
    # back substitution D L^T ct = z
    rr = np.zeros(M)
    dg = np.zeros(M)
    for (r, c, a, b), x in v.items():
        i, j = r + RI * a, c + RJ * b
        if i == M and j < M:
            rr[j] = x
        if i == j and i < M:
            dg[i] = x
    for jp in range(M - 1, -1, -1):
        cj = rr[jp] / dg[jp]
        IB = jp // RI
        r = jp - RI * IB
        for c in range(RJ):
            for b in range(bmax(RI, RJ, IB) + 1):
                j = c + RJ * b
                if j < jp:
                    assert j < M
                    rr[j] -= v[(r, c, IB, b)] * cj
        rr[jp] = cj
    return rr, np.linalg.solve(K, y)


# (RI, RJ, A, specialised steps): the layouts anchors() instantiates, and the 8 x 8 grid with 13 row blocks
LAYOUTS = [(8, 8, 7, True), (16, 16, 5, True), (16, 16, 7, True), (16, 16, 9, True), (32, 16, 7, True),
           (32, 32, 9, False), (8, 8, 13, True)]


@pytest.mark.parametrize("layout", LAYOUTS, ids=[f"{l[0]}x{l[1]}_A{l[2]}" for l in LAYOUTS])
def test_lane_logic_matches_dense_solve(layout):
    RI, RJ, A, spec = layout
    B = bmax(RI, RJ, A - 1) + 1
    nmax = min(RI * A, RJ * B)
    rng = np.random.default_rng(RI * 100 + A)
    # the largest M of the layout, a ragged one, and a small one
    for M in sorted({nmax - 1, max(2, nmax - 1 - RJ // 2 - 3), max(2, nmax // 3)}):
        got, ref = emulate(RI, RJ, A, M, rng, spec)
        assert np.allclose(got, ref, rtol=1e-10, atol=1e-12), (layout, M)
