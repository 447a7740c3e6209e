"""Helpers for the GPU parity tests: oracle-side references and tensor
conversion.  The oracle (tests' CPU reference) and the HIP library share
nothing; inputs come from `workloads`."""

import numpy as np

from oracle import fem, operators as ops

OP_NAMES = {"B0": ("B", 0.0), "BSHIFT": ("B", None), "L": ("L", None), "N": ("N", None),
            "H": ("H", None), "M": None}


def oracle_matrix(dim, n, op, k, delta_hat):
    K, M, MG = fem.assemble(dim, n)
    if op == "M":
        return M.astype(np.complex128)
    if op == "B0":
        return ops.b_delta(K, M, MG, k, 0.0).tocsr()
    if op == "BSHIFT":
        return ops.b_delta(K, M, MG, k, delta_hat).tocsr()
    if op == "L":
        return ops.hss_lhs(K, M, MG, k, delta_hat).tocsr()
    if op == "N":
        return ops.hss_rhs(K, M, MG, k, delta_hat).tocsr()
    if op == "H":
        return ops.h_gram(M, MG, k, delta_hat).tocsr().astype(np.complex128)
    raise KeyError(op)


def to_dev(a, dtype="complex128"):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to(device="cuda", dtype=getattr(torch, dtype)).contiguous()


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.complex128)


def rel_err(a, b):
    """max-norm error relative to the max-norm of the reference b."""
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def q1_rows(n, abc, ijk):
    """Rows of the 3D Q1 operator a K + b M + c M_Gamma (every face
    Sommerfeld) for the nodes ijk = [(i, j, l), ...], built one row at a
    time from the oracle's element and face matrices, so that a mesh too
    large to assemble can be checked on sampled nodes.  Returns a list of
    (columns, values)."""
    a_, b_, c_ = abc
    h = 1.0 / n
    kl, ml = fem.q1_element_matrices(h)
    gl = fem.q1_face_matrix(h)
    idx = lambda i, j, l: i + (n + 1) * (j + (n + 1) * l)
    rows = []
    for (i, j, l) in ijk:
        acc = {}
        c = (i, j, l)
        for r in (l - 1, l):
            for q in (j - 1, j):
                for p in (i - 1, i):
                    if not (0 <= p < n and 0 <= q < n and 0 <= r < n):
                        continue
                    a = (i - p) + 2 * (j - q) + 4 * (l - r)
                    for b in range(8):
                        col = idx(p + (b & 1), q + ((b >> 1) & 1), r + ((b >> 2) & 1))
                        acc[col] = acc.get(col, 0.0) + a_ * kl[a, b] + b_ * ml[a, b]
        # boundary faces: x faces span (y, z), y faces (x, z), z faces (x, y)
        for ax, (u, v) in ((0, (1, 2)), (1, (0, 2)), (2, (0, 1))):
            if c[ax] not in (0, n):
                continue
            for bv in (c[v] - 1, c[v]):
                for au in (c[u] - 1, c[u]):
                    if not (0 <= au < n and 0 <= bv < n):
                        continue
                    loc = (c[u] - au) + 2 * (c[v] - bv)
                    for m in range(4):
                        node = list(c)
                        node[u], node[v] = au + (m & 1), bv + (m >> 1)
                        col = idx(*node)
                        acc[col] = acc.get(col, 0.0) + c_ * gl[loc, m]
        cols = np.array(sorted(acc), dtype=np.int64)
        rows.append((cols, np.array([complex(acc[cc]) for cc in cols], dtype=np.complex128)))
    return rows


def q1_b0_rows(n, k, ijk):
    """Rows of B_0 = K - k^2 M - i k M_Gamma (see q1_rows)."""
    return q1_rows(n, (1.0, -k * k, -1j * k), ijk)


def row_apply(rows, x):
    """(A x) at the rows' nodes."""
    return np.array([vals @ x[cols] for cols, vals in rows])


def row_diag(rows, ijk, n):
    """The diagonal entries of the rows of nodes ijk."""
    out = []
    for (cols, vals), (i, j, l) in zip(rows, ijk):
        t = i + (n + 1) * (j + (n + 1) * l)
        out.append(vals[np.searchsorted(cols, t)])
    return np.array(out)


def q1_prolong_row(nf, node):
    """Row of the trilinear interpolation P (n/2 mesh -> nf mesh) at fine
    node (i, j, l): the coarse basis functions evaluated at the node with
    the oracle's Q1 basis.  Returns (coarse columns, weights)."""
    nc = nf // 2
    i, j, l = node
    cell = [min(v // 2, nc - 1) for v in (i, j, l)]
    loc = [v / 2.0 - cv for v, cv in zip((i, j, l), cell)]
    val, _ = fem._q1_basis(*loc)
    cols, w = [], []
    for a in range(8):
        if abs(val[a]) < 1e-14:
            continue
        I, J, L = cell[0] + (a & 1), cell[1] + ((a >> 1) & 1), cell[2] + ((a >> 2) & 1)
        cols.append(I + (nc + 1) * (J + (nc + 1) * L))
        w.append(val[a])
    return np.array(cols, dtype=np.int64), np.array(w)


def q1_restrict_rows(nf, coarse_nodes):
    """Rows of P^T at coarse nodes (I, J, L): the fine nodes within one of
    (2I, 2J, 2L) on every axis with their weights P[f, C]."""
    nc = nf // 2
    out = []
    for (I, J, L) in coarse_nodes:
        C = I + (nc + 1) * (J + (nc + 1) * L)
        fine, w = [], []
        for dl in (-1, 0, 1):
            for dj in (-1, 0, 1):
                for di in (-1, 0, 1):
                    f = (2 * I + di, 2 * J + dj, 2 * L + dl)
                    if min(f) < 0 or max(f) > nf:
                        continue
                    cols, ww = q1_prolong_row(nf, f)
                    hit = np.nonzero(cols == C)[0]
                    if hit.size:
                        fine.append(f)
                        w.append(ww[hit[0]])
        out.append((fine, np.array(w)))
    return out


def sample_nodes_3d(n, count, seed):
    """The 8 corners, one node on every edge and face, and `count` random
    nodes of the (n+1)^3 grid."""
    rng = np.random.default_rng(seed)
    pts = [(i, j, l) for i in (0, n) for j in (0, n) for l in (0, n)]
    m = n // 2
    pts += [(m, 0, 0), (0, m, n), (n, n, m), (m, m, 0), (0, m, m), (m, n, m), (n, m, m)]
    pts += [tuple(int(v) for v in rng.integers(0, n + 1, 3)) for _ in range(count)]
    return pts


def p1_b0_rows(n, k, ij):
    """Rows of the 2D P1 operator B_0 = K - k^2 M - i k M_Gamma (every side
    Sommerfeld) on the right-diagonal mesh for the nodes ij, one row at a
    time from the oracle's element matrices (see q1_b0_rows)."""
    h = 1.0 / n
    idx = lambda i, j: i + (n + 1) * j
    rows = []
    for (i, j) in ij:
        acc = {}
        for q in (j - 1, j):
            for p in (i - 1, i):
                if not (0 <= p < n and 0 <= q < n):
                    continue
                for tri in (((p, q), (p + 1, q), (p + 1, q + 1)),
                            ((p, q), (p + 1, q + 1), (p, q + 1))):
                    if (i, j) not in tri:
                        continue
                    xy = np.array([[[a * h, b * h] for a, b in tri]])
                    kl, ml = fem.p1_element_matrices(xy)
                    a = tri.index((i, j))
                    for b, (bi, bj) in enumerate(tri):
                        col = idx(bi, bj)
                        acc[col] = acc.get(col, 0.0) + kl[0, a, b] - k * k * ml[0, a, b]
        # boundary edges of length h: (h / 6) [[2, 1], [1, 2]]
        for ax in (0, 1):
            c = (i, j)
            if c[ax] not in (0, n):
                continue
            o = 1 - ax
            for e0 in (c[o] - 1, c[o]):
                if not 0 <= e0 < n:
                    continue
                for e in (e0, e0 + 1):
                    node = [0, 0]
                    node[ax], node[o] = c[ax], e
                    w = (2.0 if e == c[o] else 1.0) * h / 6.0
                    col = idx(*node)
                    acc[col] = acc.get(col, 0.0) - 1j * k * w
        cols = np.array(sorted(acc), dtype=np.int64)
        rows.append((cols, np.array([acc[cc] for cc in cols], dtype=np.complex128)))
    return rows


def sample_nodes_2d(n, count, seed):
    """The 4 corners, a node on each side, and `count` random nodes."""
    rng = np.random.default_rng(seed)
    m = n // 2
    pts = [(0, 0), (n, 0), (0, n), (n, n), (m, 0), (0, m), (n, m), (m, n)]
    pts += [tuple(int(v) for v in rng.integers(0, n + 1, 2)) for _ in range(count)]
    return pts
