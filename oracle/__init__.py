"""CPU oracle for GCA-H^2 compression of the Laplace single-layer Galerkin matrix.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the bench's CPU
baseline leg may import this package; the product library never does.  It
shares no code with the HIP library (its quadrature rules, tree construction,
cross approximation and matrix-vector product are written here independently).

Two parts:
  * O-A, the plain definition (C, FP64, ``gca_oracle.c``): every Galerkin entry
    g_ij of Eq. G_def (Section 1) by per-case quadrature (Section 8 lists the
    four Sauter cases), dense assembly, sampled rows.
  * O-B, the compression algorithm step by step (numpy, FP64), for small n:
      - cluster tree with axis-parallel bounding boxes of the supports
        (Section 2, the boxes tau and sigma containing the supports);
      - admissibility max(diam tau, diam sigma) <= 2 eta dist(tau, sigma)
        (Section 2);
      - Green quadrature points on the boundary of a box omega around tau and
        the factor A of Section 2 (entries a_{i nu}, a_{i, nu+k});
      - cross approximation of A with full pivoting, giving the pivot rows
        tau~ and V_tau with V_tau A|tau~ ~ A (Section 3);
      - nested bases: A restricted to the sons' pivots, V^_tau, transfer
        matrices E_tau1, E_tau2 (Section 4);
      - the H^2 approximation G ~ V_tau G|tau~ x sigma~ V_sigma^* on admissible
        blocks (Section 4) and G|tau^ x sigma^ on inadmissible leaf blocks,
        applied by the forward transform, coupling, backward transform and
        nearfield phases.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gca_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None

REG, NEAR, VERT, EDGE, IDENT = 0, 1, 2, 3, 4


def build() -> str:
    """Compile the C oracle (gcc -O2, no fast-math, OpenMP)."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
           "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.orc_create.restype = P
    lib.orc_create.argtypes = [I64, I64, P, P, I32, I32, I32, I32]
    lib.orc_destroy.argtypes = [P]
    lib.orc_classify.restype = I32
    lib.orc_classify.argtypes = [P, I64, I64]
    lib.orc_entry.restype = D
    lib.orc_entry.argtypes = [P, I64, I64]
    lib.orc_entries.argtypes = [P, I64, P, P, P]
    lib.orc_classify_many.argtypes = [P, I64, P, P, P]
    lib.orc_dense.argtypes = [P, P]
    lib.orc_matvec_rows.argtypes = [P, I64, P, P, I64, P]
    lib.orc_triangle_points.argtypes = [P, I32, P, P]
    lib.orc_gauss01.argtypes = [I32, P, P]
    lib.orc_tri_rule.restype = I32
    lib.orc_tri_rule.argtypes = [I32, I32, P, P, P]
    lib.orc_entry_grad.argtypes = [P, I64, I64, P]
    lib.orc_energy_grad_vertices.argtypes = [P, P, I64, P, P]
    lib.orc_num_threads.restype = I32
    lib.orc_num_threads.argtypes = []
    lib.orc_ss_moment.restype = D
    lib.orc_ss_moment.argtypes = [I32, I32, I32, I32, I32, I32]
    lib.orc_entry_dl.restype = D
    lib.orc_entry_dl.argtypes = [P, I64, I64]
    lib.orc_entries_dl.argtypes = [P, I64, P, P, P]
    lib.orc_lin_touch_moments.argtypes = [P, I64, I64, P]
    lib.orc_curved_create.restype = P
    lib.orc_curved_create.argtypes = [I64, I64, P, P, I32, I32, I32]
    lib.orc_curved_destroy.argtypes = [P]
    lib.orc_curved_classify.restype = I32
    lib.orc_curved_classify.argtypes = [P, I64, I64]
    lib.orc_curved_moments.argtypes = [P, I32, I64, I64, P]
    lib.orc_curved_moments_many.argtypes = [P, I32, I64, P, P, P]
    lib.orc_curved_mass.argtypes = [P, I64, I32, P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def gauss01(q: int):
    """Gauss-Legendre nodes and weights on [0, 1] (ascending nodes)."""
    lib = _load()
    x = np.zeros(q)
    w = np.zeros(q)
    lib.orc_gauss01(q, _ptr(x), _ptr(w))
    return x, w


def tri_rule(q: int, sym: bool = False):
    """The oracle's rule on the reference triangle {0 <= s2 <= s1 <= 1} used
    by the disjoint classes: (s1, s2, w), weights summing to 1/2."""
    n = 1024
    s1, s2, w = np.zeros(n), np.zeros(n), np.zeros(n)
    k = _load().orc_tri_rule(q, int(sym), _ptr(s1), _ptr(s2), _ptr(w))
    if k == 0:
        raise ValueError("unsupported rule")
    return s1[:k], s2[:k], w[:k]


def num_threads() -> int:
    """OpenMP threads used by the oracle's parallel loops."""
    return int(_load().orc_num_threads())


def ss_moment(kase: int, q: int, a: int, b: int, c: int, d: int) -> float:
    """Sum over the Sauter-Schwab maps of jac * x1^a x2^b y1^c y2^d."""
    return _load().orc_ss_moment(kase, q, a, b, c, d)


class Entries:
    """Galerkin entries g_ij of Eq. G_def by the oracle's quadrature rules.

    Orders: q_r (disjoint), q_nr (near-regular disjoint), q_s (touching,
    Gauss points per variable of the 4D Sauter-Schwab rules).  sym: the
    disjoint classes use the fully symmetric triangle rule of the same
    polynomial degree as the collapsed rule of their order (q = 2: 3 points,
    q = 3: 6 points) instead of the collapsed rule.
    """

    def __init__(self, verts, tris, q_r=3, q_nr=5, q_s=4, sym=False):
        self.lib = _load()
        self.verts = np.ascontiguousarray(verts, dtype=np.float64)
        self.tris = np.ascontiguousarray(tris, dtype=np.int32)
        self.n = int(self.tris.shape[0])
        self.q = (q_r, q_nr, q_s)
        self.sym = bool(sym)
        self.h = self.lib.orc_create(self.verts.shape[0], self.n, _ptr(self.verts),
                                     _ptr(self.tris), q_r, q_nr, q_s, int(self.sym))
        if not self.h:
            raise ValueError("invalid quadrature orders")

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.orc_destroy(h)
            self.h = None

    def classify(self, i, j):
        I = np.ascontiguousarray(np.atleast_1d(i), dtype=np.int64)
        J = np.ascontiguousarray(np.atleast_1d(j), dtype=np.int64)
        I, J = np.broadcast_arrays(I, J)
        I, J = np.ascontiguousarray(I), np.ascontiguousarray(J)
        out = np.zeros(I.shape, dtype=np.int32)
        self.lib.orc_classify_many(self.h, I.size, _ptr(I), _ptr(J), _ptr(out))
        return out

    def entries(self, i, j):
        I = np.ascontiguousarray(np.atleast_1d(i), dtype=np.int64)
        J = np.ascontiguousarray(np.atleast_1d(j), dtype=np.int64)
        I, J = np.broadcast_arrays(I, J)
        I, J = np.ascontiguousarray(I).ravel(), np.ascontiguousarray(J).ravel()
        out = np.zeros(I.size)
        self.lib.orc_entries(self.h, I.size, _ptr(I), _ptr(J), _ptr(out))
        return out

    def dl_entries(self, i, j):
        """Double-layer entries k_ij = int_{t_i} int_{t_j} n_j . (x - y) /
        (4 pi |x - y|^3) dy dx (n_j the unit normal of t_j), same rules per
        class as the single-layer entries; identical pairs are 0."""
        I = np.ascontiguousarray(np.atleast_1d(i), dtype=np.int64)
        J = np.ascontiguousarray(np.atleast_1d(j), dtype=np.int64)
        I, J = np.broadcast_arrays(I, J)
        I, J = np.ascontiguousarray(I).ravel(), np.ascontiguousarray(J).ravel()
        out = np.zeros(I.size)
        self.lib.orc_entries_dl(self.h, I.size, _ptr(I), _ptr(J), _ptr(out))
        return out

    def dl_block(self, rows, cols):
        rows = np.asarray(rows, dtype=np.int64)
        cols = np.asarray(cols, dtype=np.int64)
        return self.dl_entries(np.repeat(rows, cols.size), np.tile(cols, rows.size)).reshape(rows.size, cols.size)

    def lin_touch_moments(self, t, s):
        """The nine corner moments int_t int_s lambda_a g lambda_b (a, b in
        the mesh corner order of t and s) of a touching pair by the
        Sauter-Schwab maps of order q_s (Section 5's linear nodal basis)."""
        M = np.zeros(9)
        self.lib.orc_lin_touch_moments(self.h, int(t), int(s), _ptr(M))
        return M.reshape(3, 3)

    def block(self, rows, cols):
        rows = np.asarray(rows, dtype=np.int64)
        cols = np.asarray(cols, dtype=np.int64)
        I = np.repeat(rows, cols.size)
        J = np.tile(cols, rows.size)
        return self.entries(I, J).reshape(rows.size, cols.size)

    def dense(self):
        G = np.zeros((self.n, self.n))
        self.lib.orc_dense(self.h, _ptr(G))
        return G

    def matvec_rows(self, rows, x):
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        x = np.asarray(x, dtype=np.float64)
        one = x.ndim == 1
        X = np.ascontiguousarray(x.reshape(self.n, -1))
        Y = np.zeros((rows.size, X.shape[1]))
        self.lib.orc_matvec_rows(self.h, rows.size, _ptr(rows), _ptr(X), X.shape[1], _ptr(Y))
        return Y[:, 0] if one else Y

    def entry_grad(self, i, j):
        """d g_ij / d(coordinates of t_i's and t_j's vertices), shape (2, 3, 3):
        [side][vertex slot in mesh order][coordinate]; for i == j the whole
        derivative is in side 0."""
        out = np.zeros(18)
        self.lib.orc_entry_grad(self.h, int(i), int(j), _ptr(out))
        return out.reshape(2, 3, 3)

    def energy_grad_vertices(self, u, vsel):
        """dE/dX_v, E = 1/2 u^T G u, for the selected vertices (k, 3)."""
        u = np.ascontiguousarray(u, dtype=np.float64)
        vsel = np.ascontiguousarray(vsel, dtype=np.int32)
        out = np.zeros((vsel.size, 3))
        self.lib.orc_energy_grad_vertices(self.h, _ptr(u), vsel.size, _ptr(vsel), _ptr(out))
        return out

    def triangle_points(self, q):
        """Collapsed Gauss points of order q on every triangle and their weights
        (including the surface element 2|t|)."""
        P = np.zeros((self.n * q * q, 3))
        W = np.zeros(self.n * q * q)
        self.lib.orc_triangle_points(self.h, q, _ptr(P), _ptr(W))
        return P.reshape(self.n, q * q, 3), W.reshape(self.n, q * q)


# --------------------------------------------------------------------------
# O-B: the compression algorithm step by step
# --------------------------------------------------------------------------

@dataclass
class Cluster:
    begin: int
    end: int
    level: int
    sons: list = field(default_factory=list)
    lo: np.ndarray = None
    hi: np.ndarray = None
    diam: float = 0.0


@dataclass
class ClusterTree:
    perm: np.ndarray          # cluster order -> original triangle id
    nodes: list               # pre-order numbering, node 0 is the root

    def indices(self, c):
        nd = self.nodes[c]
        return self.perm[nd.begin:nd.end]

    def leaves(self):
        return [c for c, nd in enumerate(self.nodes) if not nd.sons]


def cluster_tree(verts, tris, leaf):
    """Binary cluster tree (Section 4 subdivides tau^ into two disjoint sons).

    Splitting rule: the bounding box of the triangle centroids
    ((v0 + v1) + v2) / 3 is cut along its longest axis (lowest axis on ties);
    the triangles are sorted by that centroid coordinate (ties by original
    triangle id) and the first floor(#/2) form the first son.  A cluster with
    at most `leaf` triangles is a leaf.  Bounding boxes (Section 2) enclose
    all vertices of the cluster's triangles (the supports); diam is the length
    of the box diagonal.  Nodes are numbered in pre-order.
    """
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    cent = ((verts[tris[:, 0]] + verts[tris[:, 1]]) + verts[tris[:, 2]]) / 3.0
    n = tris.shape[0]
    perm = np.arange(n, dtype=np.int64)
    nodes = []

    def rec(b, e, level):
        me = len(nodes)
        nodes.append(Cluster(b, e, level))
        idx = perm[b:e]
        vv = verts[tris[idx].ravel()]
        nodes[me].lo = vv.min(axis=0)
        nodes[me].hi = vv.max(axis=0)
        ext = nodes[me].hi - nodes[me].lo
        nodes[me].diam = math.sqrt((ext[0] * ext[0] + ext[1] * ext[1]) + ext[2] * ext[2])
        if e - b <= leaf:
            return me
        c = cent[idx]
        cext = c.max(axis=0) - c.min(axis=0)
        axis = int(np.argmax(cext))
        order = np.lexsort((idx, c[:, axis]))
        perm[b:e] = idx[order]
        mid = b + (e - b) // 2
        s1 = rec(b, mid, level + 1)
        s2 = rec(mid, e, level + 1)
        nodes[me].sons = [s1, s2]
        return me

    rec(0, n, 0)
    return ClusterTree(perm, nodes)


def box_dist(a: Cluster, b: Cluster) -> float:
    g = [max(0.0, max(b.lo[d] - a.hi[d], a.lo[d] - b.hi[d])) for d in range(3)]
    return math.sqrt((g[0] * g[0] + g[1] * g[1]) + g[2] * g[2])


def admissible(a: Cluster, b: Cluster, eta: float) -> bool:
    """max{diam tau, diam sigma} <= 2 eta dist(tau, sigma) (Section 2); blocks at
    distance zero are never admissible."""
    d = box_dist(a, b)
    return d > 0.0 and max(a.diam, b.diam) <= 2.0 * eta * d


def block_tree(tree: ClusterTree, eta: float):
    """Block partition of I x I: admissible blocks (far) and inadmissible leaf
    blocks (near).  Recursion from (root, root); a non-admissible block with a
    non-leaf member is split into the sons of every non-leaf member."""
    far, near = [], []
    stack = [(0, 0)]
    while stack:
        t, s = stack.pop()
        nt, ns = tree.nodes[t], tree.nodes[s]
        if admissible(nt, ns, eta):
            far.append((t, s))
            continue
        if not nt.sons and not ns.sons:
            near.append((t, s))
            continue
        ts = nt.sons if nt.sons else [t]
        ss = ns.sons if ns.sons else [s]
        for a in ts:
            for b in ss:
                stack.append((a, b))
    far.sort()
    near.sort()
    return far, near


def green_points(c: Cluster, m: int, eta: float, omega_scale: float = 0.25):
    """Green quadrature for the box omega = [lo - delta, hi + delta], delta =
    omega_scale * diam / eta (Section 2: a superset omega of tau whose boundary
    keeps a distance from tau).  On each of the six faces a tensor m x m
    Gauss-Legendre rule; outward unit normals.  Returns (z (k,3), w (k,),
    n (k,3)) with k = 6 m^2, faces ordered (axis 0 low, axis 0 high, axis 1
    low, ...), points on a face ordered by the lower remaining axis first."""
    x, w = gauss01(m)
    delta = omega_scale * c.diam / eta
    L = c.lo - delta
    H = c.hi + delta
    Z, W, N = [], [], []
    for a in range(3):
        b, cc = [d for d in range(3) if d != a]
        for side in (-1, 1):
            for i in range(m):
                for j in range(m):
                    z = np.zeros(3)
                    z[a] = L[a] if side < 0 else H[a]
                    z[b] = L[b] + x[i] * (H[b] - L[b])
                    z[cc] = L[cc] + x[j] * (H[cc] - L[cc])
                    nv = np.zeros(3)
                    nv[a] = float(side)
                    Z.append(z)
                    W.append(w[i] * w[j] * (H[b] - L[b]) * (H[cc] - L[cc]))
                    N.append(nv)
    return np.array(Z), np.array(W), np.array(N)


def green_factor_A(rows, tri_pts, tri_wts, z, wz, nz, diam):
    """A in R^{rows x 2k} of Section 2:
        a_{i nu}     =  sqrt(w_nu) int g(x, z_nu) phi_i(x) dx
        a_{i, nu+k}  = -d_tau sqrt(w_nu) int dg/dn_z(x, z_nu) phi_i(x) dx
    with dg/dn_z(x, z) = n_z . (x - z) / (4 pi |x - z|^3)."""
    P = tri_pts[rows]                 # (r, p, 3)
    Wt = tri_wts[rows]                # (r, p)
    d = P[:, :, None, :] - z[None, None, :, :]        # x - z, (r, p, k, 3)
    r = np.sqrt(np.sum(d * d, axis=-1))
    g = 1.0 / (4.0 * math.pi * r)
    dg = np.einsum("rpkd,kd->rpk", d, nz) / (4.0 * math.pi * r ** 3)
    sw = np.sqrt(wz)
    A1 = sw[None, :] * np.einsum("rp,rpk->rk", Wt, g)
    A2 = -diam * sw[None, :] * np.einsum("rp,rpk->rk", Wt, dg)
    return np.concatenate([A1, A2], axis=1)


def aca_full(A, eps):
    """Cross approximation with full pivoting (Section 3: the thin A allows a
    reliable pivoting strategy).  R <- A; while ||R||_F > eps ||A||_F and
    r < min(rows, cols): (p, q) = argmax |R| (first in row-major order, i.e.
    smallest row then smallest column on ties); stop if R_pq = 0;
    R <- R - R[:, q] R[p, :] / R_pq.  Returns pivot rows I, pivot columns J
    and V = A[:, J] A[I, J]^{-1} with rows I set to the identity (the
    interpolation property V A|I = A on the pivot rows)."""
    A = np.asarray(A, dtype=np.float64)
    R = A.copy()
    nA = np.linalg.norm(A)
    I, J = [], []
    rmax = min(A.shape)
    while len(I) < rmax:
        if np.linalg.norm(R) <= eps * nA:
            break
        flat = int(np.argmax(np.abs(R)))
        p, q = divmod(flat, R.shape[1])
        piv = R[p, q]
        if piv == 0.0:
            break
        R = R - np.outer(R[:, q], R[p, :]) / piv
        I.append(p)
        J.append(q)
    if not I:
        return np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.int64), np.zeros((A.shape[0], 0))
    I = np.array(I, dtype=np.int64)
    J = np.array(J, dtype=np.int64)
    V = np.linalg.solve(A[np.ix_(I, J)].T, A[:, J].T).T
    V[I, :] = np.eye(len(I))
    return I, J, V


@dataclass
class H2:
    tree: ClusterTree
    far: list
    near: list
    pivots: dict       # cluster -> original triangle ids tau~ (pivot order)
    V: dict            # leaf -> V_tau (|tau^| x |tau~|), rows in cluster order
    E: dict            # non-root cluster -> E_tau (|tau~| x |parent~|)
    ent: Entries
    blocks: dict = field(default_factory=dict)   # entries of coupling / near blocks, filled on first use
    ent_c: Entries = None                        # rule of the coupling entries (default: ent)

    def coupling(self, t, s):
        key = ("far", t, s)
        if key not in self.blocks:
            e = self.ent_c if self.ent_c is not None else self.ent
            self.blocks[key] = e.block(self.pivots[t], self.pivots[s])
        return self.blocks[key]

    def nearblock(self, t, s):
        key = ("near", t, s)
        if key not in self.blocks:
            self.blocks[key] = self.ent.block(self.tree.indices(t), self.tree.indices(s))
        return self.blocks[key]


def gca_h2(verts, tris, leaf=32, eta=2.0, m=3, eps=1e-6, q_A=3, q=(3, 5, 4),
           omega_scale=0.25, ent=None, q_c=None):
    """Build the GCA-H^2 approximation step by step (Sections 2-4).  q_c: order
    of the regular rule for the coupling entries G|t~ x s~ (default q[0]); the
    coupling matrices are Galerkin entries of well-separated pairs, whose
    rule order is a parameter of the method like the others, and it applies
    to every pivot pair of an admissible block."""
    tree = cluster_tree(verts, tris, leaf)
    far, near = block_tree(tree, eta)
    if ent is None:
        ent = Entries(verts, tris, *q)
    tp, tw = ent.triangle_points(q_A)
    pivots, V, E = {}, {}, {}
    # post-order over the pre-order numbering: sons have larger numbers
    for c in reversed(range(len(tree.nodes))):
        nd = tree.nodes[c]
        z, wz, nz = green_points(nd, m, eta, omega_scale)
        if not nd.sons:
            rows = tree.indices(c)
        else:
            rows = np.concatenate([pivots[s] for s in nd.sons])
        A = green_factor_A(rows, tp, tw, z, wz, nz, nd.diam)
        I, _, Vh = aca_full(A, eps)
        pivots[c] = rows[I]
        if not nd.sons:
            V[c] = Vh
        else:
            o = 0
            for s in nd.sons:
                r = len(pivots[s])
                E[s] = Vh[o:o + r, :]
                o += r
    # the coupling entries are entries of admissible blocks: one regular rule
    # of order q_c for every pivot pair, also for a pair whose vertices are
    # joined by an edge (the near-regular order is a nearfield refinement)
    qc = q[0] if q_c is None else q_c
    ent_c = None
    if qc != q[0] or q[1] != qc:
        ent_c = Entries(verts, tris, qc, qc, q[2], sym=ent.sym)
    return H2(tree, far, near, pivots, V, E, ent, ent_c=ent_c)


def h2_matvec(h: H2, x):
    """y = G~ x by the four H^2 phases: forward transform (leaf V^T, then E^T
    upwards), coupling with the original entries G|tau~ x sigma~, backward
    transform (E downwards, leaf V), and the inadmissible leaf blocks."""
    tree, ent = h.tree, h.ent
    x = np.asarray(x, dtype=np.float64)
    X = x.reshape(x.shape[0], -1)
    nn = len(tree.nodes)
    xh = [None] * nn
    for c in reversed(range(nn)):
        nd = tree.nodes[c]
        if not nd.sons:
            xh[c] = h.V[c].T @ X[tree.indices(c)]
        else:
            xh[c] = sum(h.E[s].T @ xh[s] for s in nd.sons)
    yh = [np.zeros((len(h.pivots[c]), X.shape[1])) for c in range(nn)]
    for (t, s) in h.far:
        yh[t] += h.coupling(t, s) @ xh[s]
    Y = np.zeros_like(X)
    for c in range(nn):
        nd = tree.nodes[c]
        for s in nd.sons:
            yh[s] += h.E[s] @ yh[c]
        if not nd.sons:
            Y[tree.indices(c)] += h.V[c] @ yh[c]
    for (t, s) in h.near:
        rows, cols = tree.indices(t), tree.indices(s)
        Y[rows] += h.nearblock(t, s) @ X[cols]
    return Y.reshape(x.shape)


def expanded_basis(h: H2, c):
    """V_tau written out: the leaf basis, or diag(V_tau1 E_tau1, V_tau2 E_tau2)
    stacked for the sons (Section 4); rows in cluster order of tau^."""
    nd = h.tree.nodes[c]
    if not nd.sons:
        return h.V[c]
    return np.concatenate([expanded_basis(h, s) @ h.E[s] for s in nd.sons], axis=0)


def h2_dense(h: H2):
    """The H^2 approximation as an explicit n x n matrix:
    V_tau G|tau~ x sigma~ V_sigma^T on admissible blocks, G|tau^ x sigma^ on
    inadmissible leaf blocks."""
    n = len(h.tree.perm)
    Gt = np.zeros((n, n))
    cache = {}
    for (t, s) in h.far:
        for c in (t, s):
            if c not in cache:
                cache[c] = expanded_basis(h, c)
        Gt[np.ix_(h.tree.indices(t), h.tree.indices(s))] = cache[t] @ h.coupling(t, s) @ cache[s].T
    for (t, s) in h.near:
        Gt[np.ix_(h.tree.indices(t), h.tree.indices(s))] = h.nearblock(t, s)
    return Gt


def spectral_norm_sym(apply, n, iters=30, seed=0):
    """Power iteration estimate of the spectral norm of a symmetric operator
    (Section 2 estimates relative spectral errors this way)."""
    v = np.random.default_rng(seed).standard_normal(n)
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = apply(v)
        lam = np.linalg.norm(w)
        if lam == 0.0:
            return 0.0
        v = w / lam
    return lam
