"""Meshes, element matrices and global assembly for the primal form (Sec. 2).

The primal form of the paper (Sec. 2, eq. (primal)) is

    b_delta(u, v) = int (-delta + i k)^2 u v* + grad u . grad v*
                    - (-delta + i k) int_Gamma u v*,

discretised with continuous piecewise-linear (CG1) functions.  With a real
nodal basis {phi_i} every matrix the method needs is a complex combination
of three real symmetric matrices, assembled here element by element:

    K_ij  = int grad phi_j . grad phi_i       (stiffness)
    M_ij  = int phi_j phi_i                   (mass)
    MG_ij = int_Gamma phi_j phi_i             (boundary mass on Gamma)

Meshes are uniform on the unit square / cube, n cells per side.
  * 2D: every cell [x_p, x_p+1] x [y_q, y_q+1] is split along its diagonal
    from (x_p, y_q) to (x_p+1, y_q+1) into two P1 triangles (the "right
    diagonal" reading of the paper's uniformly triangular mesh).
  * 3D: Q1 hexahedra (trilinear), the element the benchmark workloads name.
Nodes are numbered lexicographically, node (i, j[, l]) has index
i + (n+1) * (j + (n+1) * l), coordinates (i/n, j/n[, l/n]).

Nothing here is specialised to a stencil: local matrices come from vertex
coordinates (P1) or Gauss quadrature (Q1) and are scattered into COO form.
"""

import numpy as np
import scipy.sparse as sp

FACES_2D = ("x0", "x1", "y0", "y1")
FACES_3D = ("x0", "x1", "y0", "y1", "z0", "z1")


# ---------------------------------------------------------------- 2D, P1 ---

def nodes_2d(n):
    """Coordinates (N, 2) of the (n+1)^2 nodes, lexicographic (i fastest)."""
    t = np.arange(n + 1) / n
    X, Y = np.meshgrid(t, t, indexing="xy")  # X[j, i] = x_i
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def triangles_2d(n):
    """Connectivity (2 n^2, 3) of the right-diagonal triangulation.

    Cell (p, q) gives the triangles {(p,q), (p+1,q), (p+1,q+1)} and
    {(p,q), (p+1,q+1), (p,q+1)}; both contain the cell diagonal.
    """
    def idx(i, j):
        return i + (n + 1) * j
    p, q = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    p, q = p.ravel(), q.ravel()
    t1 = np.stack([idx(p, q), idx(p + 1, q), idx(p + 1, q + 1)], axis=1)
    t2 = np.stack([idx(p, q), idx(p + 1, q + 1), idx(p, q + 1)], axis=1)
    return np.concatenate([t1, t2], axis=0)


def p1_element_matrices(xy):
    """Local P1 stiffness and mass for triangles with vertices xy (E, 3, 2).

    The barycentric gradients follow from the affine map
    x = x0 + B (s, t); the mass uses the exact P1 formula
    int phi_a phi_b = |T| (1 + [a == b]) / 12.
    """
    B = np.stack([xy[:, 1] - xy[:, 0], xy[:, 2] - xy[:, 0]], axis=2)  # (E,2,2)
    area = 0.5 * np.abs(np.linalg.det(B))
    gref = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])  # d phi / d(s,t)
    binv = np.linalg.inv(B)                                   # d(s,t) / dx
    grad = np.einsum("as,est->eat", gref, binv)               # (E,3,2)
    kloc = area[:, None, None] * np.einsum("eat,ebt->eab", grad, grad)
    mloc = (area[:, None, None] / 12.0) * (np.ones((3, 3)) + np.eye(3))[None]
    return kloc, mloc


def boundary_edges_2d(n, faces=FACES_2D):
    """Boundary edges (node pairs) lying on the requested faces of the square."""
    def idx(i, j):
        return i + (n + 1) * j
    r = np.arange(n)
    out = []
    if "y0" in faces:
        out.append(np.stack([idx(r, 0), idx(r + 1, 0)], axis=1))
    if "y1" in faces:
        out.append(np.stack([idx(r, n), idx(r + 1, n)], axis=1))
    if "x0" in faces:
        out.append(np.stack([idx(0, r), idx(0, r + 1)], axis=1))
    if "x1" in faces:
        out.append(np.stack([idx(n, r), idx(n, r + 1)], axis=1))
    if not out:
        return np.zeros((0, 2), dtype=np.int64)
    return np.concatenate(out, axis=0)


def _scatter(conn, local, size):
    nloc = conn.shape[1]
    rows = np.repeat(conn, nloc, axis=1).ravel()
    cols = np.tile(conn, (1, nloc)).ravel()
    return sp.coo_matrix((local.ravel(), (rows, cols)), shape=(size, size)).tocsr()


def assemble_2d(n, faces=FACES_2D):
    """Assemble (K, M, MG) for P1 on the right-diagonal n x n mesh.

    MG integrates over the boundary edges on the faces listed in `faces`
    (the Sommerfeld part Gamma of the boundary); each edge of length l
    contributes (l / 6) [[2, 1], [1, 2]].
    """
    xy = nodes_2d(n)
    tri = triangles_2d(n)
    kloc, mloc = p1_element_matrices(xy[tri])
    size = xy.shape[0]
    K = _scatter(tri, kloc, size)
    M = _scatter(tri, mloc, size)
    edges = boundary_edges_2d(n, faces)
    length = np.linalg.norm(xy[edges[:, 1]] - xy[edges[:, 0]], axis=1)
    gloc = (length[:, None, None] / 6.0) * np.array([[2.0, 1.0], [1.0, 2.0]])[None]
    MG = _scatter(edges, gloc, size)
    return K, M, MG


def locate_p1_2d(nc, pts):
    """Barycentric weights of points in the coarse right-diagonal mesh.

    Returns (nodes (P, 3), weights (P, 3)) with coarse node indices of the
    triangle containing each point.  Points on shared edges may be assigned
    to either neighbour; the interpolant is continuous so the value agrees.
    """
    hc = 1.0 / nc
    p = np.clip(np.floor(pts[:, 0] / hc + 1e-12).astype(np.int64), 0, nc - 1)
    q = np.clip(np.floor(pts[:, 1] / hc + 1e-12).astype(np.int64), 0, nc - 1)
    s = pts[:, 0] / hc - p
    t = pts[:, 1] / hc - q
    lower = t <= s + 1e-12  # below the diagonal: triangle (p,q),(p+1,q),(p+1,q+1)

    def idx(i, j):
        return i + (nc + 1) * j
    nodes = np.where(
        lower[:, None],
        np.stack([idx(p, q), idx(p + 1, q), idx(p + 1, q + 1)], axis=1),
        np.stack([idx(p, q), idx(p + 1, q + 1), idx(p, q + 1)], axis=1),
    )
    # barycentric coordinates from the vertex coordinates
    cxy = nodes_2d(nc)[nodes]  # (P,3,2)
    B = np.stack([cxy[:, 1] - cxy[:, 0], cxy[:, 2] - cxy[:, 0]], axis=2)
    st = np.linalg.solve(B, (pts - cxy[:, 0])[:, :, None])[:, :, 0]
    w = np.stack([1.0 - st[:, 0] - st[:, 1], st[:, 0], st[:, 1]], axis=1)
    return nodes, w


def prolongation_2d(nf):
    """Interpolation matrix P (fine x coarse) from the n/2 mesh to the n mesh.

    P_ij = phi^coarse_j(x^fine_i): the standard finite-element transfer
    between nested CG1 spaces (the paper's "standard transfer operators").
    Restriction is P^T.
    """
    assert nf % 2 == 0
    nc = nf // 2
    pts = nodes_2d(nf)
    nodes, w = locate_p1_2d(nc, pts)
    rows = np.repeat(np.arange(pts.shape[0]), 3)
    P = sp.coo_matrix((w.ravel(), (rows, nodes.ravel())),
                      shape=(pts.shape[0], (nc + 1) ** 2)).tocsr()
    P.data[np.abs(P.data) < 1e-14] = 0.0
    P.eliminate_zeros()
    return P


def boundary_node_mask_2d(n):
    i, j = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    return ((i == 0) | (i == n) | (j == 0) | (j == n)).ravel()


# ---------------------------------------------------------------- 3D, Q1 ---

def nodes_3d(n):
    t = np.arange(n + 1) / n
    Z, Y, X = np.meshgrid(t, t, t, indexing="ij")  # X[l, j, i] = x_i
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


_GAUSS2 = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))  # on [0, 1]


def _q1_basis(xi, eta, zeta):
    """Trilinear basis values and reference gradients at one point.

    Local node a = a0 + 2 a1 + 4 a2 sits at reference corner (a0, a1, a2).
    """
    lin = lambda s, a: s if a else 1.0 - s
    dlin = lambda a: 1.0 if a else -1.0
    val = np.zeros(8)
    grad = np.zeros((8, 3))
    for a in range(8):
        a0, a1, a2 = a & 1, (a >> 1) & 1, (a >> 2) & 1
        val[a] = lin(xi, a0) * lin(eta, a1) * lin(zeta, a2)
        grad[a] = (dlin(a0) * lin(eta, a1) * lin(zeta, a2),
                   lin(xi, a0) * dlin(a1) * lin(zeta, a2),
                   lin(xi, a0) * lin(eta, a1) * dlin(a2))
    return val, grad


def q1_element_matrices(h):
    """Q1 stiffness and mass of a cube of side h by 2x2x2 Gauss quadrature
    (exact for trilinear products)."""
    kloc = np.zeros((8, 8))
    mloc = np.zeros((8, 8))
    for xi in _GAUSS2:
        for eta in _GAUSS2:
            for zeta in _GAUSS2:
                val, grad = _q1_basis(xi, eta, zeta)
                wq = 0.125  # product of the three 1D weights on [0, 1]
                kloc += wq * (grad @ grad.T) * h   # (1/h^2) * h^3
                mloc += wq * np.outer(val, val) * h ** 3
    return kloc, mloc


def q1_face_matrix(h):
    """Bilinear face mass of a square face of side h (2x2 Gauss)."""
    g = np.zeros((4, 4))
    for s in _GAUSS2:
        for t in _GAUSS2:
            v = np.array([(1 - s) * (1 - t), s * (1 - t), (1 - s) * t, s * t])
            g += 0.25 * np.outer(v, v) * h * h
    return g


def hexes_3d(n):
    def idx(i, j, l):
        return i + (n + 1) * (j + (n + 1) * l)
    r, q, p = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    p, q, r = p.ravel(), q.ravel(), r.ravel()
    cols = []
    for a in range(8):
        a0, a1, a2 = a & 1, (a >> 1) & 1, (a >> 2) & 1
        cols.append(idx(p + a0, q + a1, r + a2))
    return np.stack(cols, axis=1)


def boundary_faces_3d(n, faces=FACES_3D):
    """Boundary quads (F, 4), local order (s,t) = (0,0),(1,0),(0,1),(1,1)."""
    def idx(i, j, l):
        return i + (n + 1) * (j + (n + 1) * l)
    b, a = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    a, b = a.ravel(), b.ravel()
    out = []
    for face in faces:
        fixed = 0 if face[1] == "0" else n
        if face[0] == "x":
            f = lambda s, t: idx(fixed, a + s, b + t)
        elif face[0] == "y":
            f = lambda s, t: idx(a + s, fixed, b + t)
        else:
            f = lambda s, t: idx(a + s, b + t, fixed)
        out.append(np.stack([f(0, 0), f(1, 0), f(0, 1), f(1, 1)], axis=1))
    if not out:
        return np.zeros((0, 4), dtype=np.int64)
    return np.concatenate(out, axis=0)


def assemble_3d(n, faces=FACES_3D):
    """Assemble (K, M, MG) for Q1 on the uniform n^3 hexahedral mesh."""
    h = 1.0 / n
    hexes = hexes_3d(n)
    kloc, mloc = q1_element_matrices(h)
    size = (n + 1) ** 3
    E = hexes.shape[0]
    K = _scatter(hexes, np.broadcast_to(kloc, (E, 8, 8)), size)
    M = _scatter(hexes, np.broadcast_to(mloc, (E, 8, 8)), size)
    quads = boundary_faces_3d(n, faces)
    gloc = q1_face_matrix(h)
    MG = _scatter(quads, np.broadcast_to(gloc, (quads.shape[0], 4, 4)), size)
    return K, M, MG


def prolongation_3d(nf):
    """Trilinear interpolation from the n/2 hexahedral mesh to the n mesh."""
    assert nf % 2 == 0
    nc = nf // 2
    pts = nodes_3d(nf)
    hc = 1.0 / nc
    cell = np.clip(np.floor(pts / hc + 1e-12).astype(np.int64), 0, nc - 1)
    loc = pts / hc - cell
    rows, cols, vals = [], [], []
    for a in range(8):
        a0, a1, a2 = a & 1, (a >> 1) & 1, (a >> 2) & 1
        w = ((loc[:, 0] if a0 else 1 - loc[:, 0])
             * (loc[:, 1] if a1 else 1 - loc[:, 1])
             * (loc[:, 2] if a2 else 1 - loc[:, 2]))
        c = (cell[:, 0] + a0) + (nc + 1) * ((cell[:, 1] + a1) + (nc + 1) * (cell[:, 2] + a2))
        rows.append(np.arange(pts.shape[0]))
        cols.append(c)
        vals.append(w)
    P = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(pts.shape[0], (nc + 1) ** 3)).tocsr()
    P.data[np.abs(P.data) < 1e-14] = 0.0
    P.eliminate_zeros()
    return P


# ------------------------------------------------------------- dispatch ---

def assemble(dim, n, faces=None):
    if dim == 2:
        return assemble_2d(n, FACES_2D if faces is None else faces)
    if dim == 3:
        return assemble_3d(n, FACES_3D if faces is None else faces)
    raise ValueError("dim must be 2 or 3")


def prolongation(dim, nf):
    return prolongation_2d(nf) if dim == 2 else prolongation_3d(nf)


def nodes(dim, n):
    return nodes_2d(n) if dim == 2 else nodes_3d(n)


def dirichlet_node_mask(dim, n, dirichlet):
    """True at the nodes lying on any of the faces named in `dirichlet`
    ("x0" is the face x = 0, "x1" the face x = 1, and so on)."""
    names = FACES_2D if dim == 2 else FACES_3D
    for f in dirichlet:
        if f not in names:
            raise ValueError("unknown face " + repr(f))
    X = nodes(dim, n)
    mask = np.zeros(X.shape[0], dtype=bool)
    for f in dirichlet:
        ax = "xyz".index(f[0])
        mask |= np.isclose(X[:, ax], 0.0 if f[1] == "0" else 1.0)
    return mask


def impedance_faces(dim, dirichlet):
    """The faces that keep the boundary (impedance) term when the faces in
    `dirichlet` carry u = 0 instead: the rest of the boundary."""
    names = FACES_2D if dim == 2 else FACES_3D
    return tuple(f for f in names if f not in dirichlet)


def eliminate(A, mask):
    """Homogeneous Dirichlet conditions by elimination: the nodes in `mask`
    leave the unknowns, so their rows and columns are removed from A and,
    to keep one index per node, replaced by those of the identity.  The
    system A' x = b with b = 0 on those nodes then has x = 0 there and the
    reduced system on the other nodes."""
    keep = sp.diags((~mask).astype(np.float64))
    return (keep @ A @ keep + sp.diags(mask.astype(np.float64))).tocsr()


def restrict_prolongation(P, fine_mask, coarse_mask):
    """Interpolation between the spaces with the Dirichlet nodes removed:
    P with the rows of fine Dirichlet nodes and the columns of coarse
    Dirichlet nodes set to zero."""
    return (sp.diags((~fine_mask).astype(np.float64)) @ P
            @ sp.diags((~coarse_mask).astype(np.float64))).tocsr()


# ----------------------------------------------- quadrature load vectors ---

def _gauss01(q):
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def load_vector_2d(n, f, g=None, q=6, faces=FACES_2D):
    """b_i = int f phi_i + int_Gamma g phi_i on the right-diagonal P1 mesh.

    Volume integrals use a collapsed (Duffy) q x q Gauss product rule on each
    triangle, edge integrals q-point Gauss.  f and g are callables of
    (x, y) arrays; g may also take the outward normal (nx, ny).  Used for
    manufactured-solution checks of the assembly (the boundary term carries
    inhomogeneous Sommerfeld data, which the paper's problem sets to zero).
    """
    xy = nodes_2d(n)
    tri = triangles_2d(n)
    v = xy[tri]                       # (E,3,2)
    s1, w1 = _gauss01(q)
    S, T = np.meshgrid(s1, s1, indexing="ij")
    W = np.outer(w1, w1)
    # reference triangle point: (s, t(1-s)), Jacobian (1 - s)
    rs, rt, rw = S.ravel(), (T * (1 - S)).ravel(), (W * (1 - S)).ravel()
    lam = np.stack([1 - rs - rt, rs, rt], axis=1)           # (Q,3) barycentric
    B = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]], axis=2)
    det = np.abs(np.linalg.det(B))                           # 2 |T|
    pts = v[:, 0][:, None, :] + np.einsum("eij,qj->eqi", B, np.stack([rs, rt], 1))
    fv = f(pts[..., 0], pts[..., 1])                         # (E,Q)
    contrib = np.einsum("eq,qa,q->ea", fv, lam, rw) * det[:, None]
    b = np.zeros(xy.shape[0], dtype=np.complex128)
    np.add.at(b, tri.ravel(), contrib.ravel())
    if g is not None:
        for face in faces:
            edges = boundary_edges_2d(n, (face,))
            a, c = xy[edges[:, 0]], xy[edges[:, 1]]
            length = np.linalg.norm(c - a, axis=1)
            normal = {"x0": (-1.0, 0.0), "x1": (1.0, 0.0),
                      "y0": (0.0, -1.0), "y1": (0.0, 1.0)}[face]
            p = a[:, None, :] + s1[None, :, None] * (c - a)[:, None, :]
            gv = g(p[..., 0], p[..., 1], normal)              # (F,q)
            ca = np.einsum("fq,q->f", gv * (1 - s1)[None], w1) * length
            cb = np.einsum("fq,q->f", gv * s1[None], w1) * length
            np.add.at(b, edges[:, 0], ca)
            np.add.at(b, edges[:, 1], cb)
    return b


def load_vector_3d(n, f, g=None, q=3, faces=FACES_3D):
    """3D Q1 counterpart of `load_vector_2d` (tensor Gauss rules)."""
    h = 1.0 / n
    hexes = hexes_3d(n)
    xyz = nodes_3d(n)
    s1, w1 = _gauss01(q)
    b = np.zeros(xyz.shape[0], dtype=np.complex128)
    origin = xyz[hexes[:, 0]]
    for i, (xi, wx) in enumerate(zip(s1, w1)):
        for (eta, wy) in zip(s1, w1):
            for (zeta, wz) in zip(s1, w1):
                val, _ = _q1_basis(xi, eta, zeta)
                p = origin + h * np.array([xi, eta, zeta])
                fv = f(p[:, 0], p[:, 1], p[:, 2]) * (wx * wy * wz * h ** 3)
                np.add.at(b, hexes.ravel(), (fv[:, None] * val[None, :]).ravel())
    if g is not None:
        for face in faces:
            quads = boundary_faces_3d(n, (face,))
            axis = "xyz".index(face[0])
            normal = np.zeros(3)
            normal[axis] = -1.0 if face[1] == "0" else 1.0
            o = xyz[quads[:, 0]]
            tang = [d for d in range(3) if d != axis]
            for (s, ws) in zip(s1, w1):
                for (t, wt) in zip(s1, w1):
                    p = o.copy()
                    p[:, tang[0]] += h * s
                    p[:, tang[1]] += h * t
                    gv = g(p[:, 0], p[:, 1], p[:, 2], tuple(normal)) * (ws * wt * h * h)
                    vals = np.array([(1 - s) * (1 - t), s * (1 - t), (1 - s) * t, s * t])
                    np.add.at(b, quads.ravel(), (gv[:, None] * vals[None, :]).ravel())
    return b
