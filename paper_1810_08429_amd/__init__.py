"""Python binding of libgca (argument marshalling only; every step of the
compression and of the matrix-vector product runs in the HIP library).

    import paper_1810_08429_amd as gca
    tree = gca.Tree(verts, tris, leaf=64)
    H = gca.H2(verts, tris, tree, gca.Params(eta=2.0, eps=1e-4))
    y = H.matvec(x)                       # x: torch cuda float64 or float32, original order
    y = H.matvec(x, precision=gca.MIXED)

PyTorch supplies device memory and the stream: vectors are tensors, the
stream is torch.cuda.current_stream(), and the library's own device memory
comes from torch's caching allocator through the gca_params callbacks
(Params(allocator=None) selects hipMalloc instead).  The library must be
built first (python -m paper_1810_08429_amd.build); importing never falls
back to anything else.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgca.so")

FP64, MIXED = 0, 1
F64, F32 = 0, 1          # gca_dtype of the vectors of h2_matvec
PHASES = ["permute", "forward", "coupling_blocks", "coupling_reduce", "backward", "near_blocks",
          "near_regular", "touching", "gather", "total"]
STATUS = {0: "GCA_OK", -1: "GCA_EINVAL", -2: "GCA_ENOMEM", -3: "GCA_EHIP", -4: "GCA_EMESH",
          -5: "GCA_ENOTSPD", -6: "GCA_ENOCONV", -7: "GCA_EINTERNAL"}

EXPORTED = [
    "gca_params_default", "gca_tree_build", "gca_tree_info", "gca_tree_export", "gca_tree_destroy",
    "gca_block_tree",
    "gca_build", "h2_matvec", "gca_entries", "gca_basis_sizes", "gca_basis_export", "gca_stats",
    "gca_destroy", "gca_last_error", "gca_phase_times", "gca_solve_refined", "gca_update_geometry",
    "h2_bilinear_grad", "gca_store_blocks", "gca_energy", "gca_energy_noalloc",
    "gca_block_entries", "gca_dl_entries",
    "gca_lin_vertex_triangles", "gca_lin_merge", "gca_lin_blocks", "gca_coll_blocks",
    "gca_curved_entries", "gca_lin_build", "gca_lin_matvec", "gca_lin_info", "gca_lin_export", "gca_lin_destroy",
]


class Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.msg = msg


class _Mesh(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int64), ("nt", ctypes.c_int64),
                ("xyz", ctypes.c_void_p), ("tri", ctypes.c_void_p)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class _Params(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("eps", ctypes.c_double), ("omega_scale", ctypes.c_double),
                ("green_m", ctypes.c_int32), ("q_A", ctypes.c_int32), ("q_r", ctypes.c_int32),
                ("q_nr", ctypes.c_int32), ("q_s", ctypes.c_int32), ("q_c", ctypes.c_int32),
                ("sym_rules", ctypes.c_int32), ("ss_fp32", ctypes.c_int32), ("serial", ctypes.c_int32),
                ("alloc", _ALLOC_FN), ("free", _FREE_FN), ("alloc_ctx", ctypes.c_void_p)]


def _torch_alloc(nbytes, stream, ctx):
    """gca_alloc_fn: a block of torch's caching allocator on the call's stream."""
    import torch
    return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))


def _torch_free(ptr, stream, ctx):
    """gca_free_fn: returns a block to torch's caching allocator."""
    import torch
    torch.cuda.caching_allocator_delete(int(ptr))


_TORCH_ALLOC = _ALLOC_FN(_torch_alloc)
_TORCH_FREE = _FREE_FN(_torch_free)


class _Stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "n", "nv", "n_clusters", "n_leaves", "depth", "n_far", "n_near", "n_far_sym", "n_near_sym",
        "n_ident", "n_edge", "n_vert", "n_nearreg", "coupling_entries", "near_pairs", "near_regular_pairs",
        "rank_min",
        "rank_max")] + [("rank_mean", ctypes.c_double), ("basis_bytes_fp64", ctypes.c_int64),
                        ("build_ms", ctypes.c_double), ("setup_ms", ctypes.c_double * 8),
                        ("phase_ms", ctypes.c_double * 10), ("store_entries_far", ctypes.c_int64),
                        ("store_entries_near", ctypes.c_int64), ("stored_mask", ctypes.c_int32),
                        ("reserved_i", ctypes.c_int32),
                        ("basis_entries_leaf", ctypes.c_int64), ("basis_entries_transfer", ctypes.c_int64)]


_lib = None


def lib():
    """The loaded libgca.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1810_08429_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.gca_params_default.argtypes = [P]
    L.gca_params_default.restype = None
    L.gca_tree_build.argtypes = [P, I32, P]
    L.gca_tree_info.argtypes = [P, P, P]
    L.gca_tree_export.argtypes = [P, P, P, P]
    L.gca_block_tree.argtypes = [P, D, I64, P, P, I64, P, P]
    L.gca_tree_destroy.argtypes = [P]
    L.gca_tree_destroy.restype = None
    L.gca_build.argtypes = [P, P, P, P, P]
    L.h2_matvec.argtypes = [P, P, P, I64, I64, I32, I32, P]
    L.gca_energy.argtypes = [P, P, P, P, P, I32, P]
    L.gca_energy_noalloc.argtypes = [P, P, P, P, P, I32, P]
    L.gca_block_entries.argtypes = [P, I32, I32, I64, P, P, P, P, P]
    L.gca_dl_entries.argtypes = [P, P, P, I64, P, P]
    L.gca_entries.argtypes = [P, P, P, I64, P, I32, P]
    L.gca_basis_sizes.argtypes = [P, P, P]
    L.gca_basis_export.argtypes = [P, P, P, P]
    L.gca_stats.argtypes = [P, P]
    L.gca_update_geometry.argtypes = [P, P, P]
    L.h2_bilinear_grad.argtypes = [P, P, P, D, P, P, I32, P]
    L.gca_solve_refined.argtypes = [P, P, P, D, I32, D, I32, P, P, P]
    L.gca_phase_times.argtypes = [P, I64, P, P]
    L.gca_store_blocks.argtypes = [P, I32, P]
    L.gca_lin_vertex_triangles.argtypes = [P, I64, I64, P, P]
    L.gca_lin_merge.argtypes = [P, P, P, P, P, I32, I32, P, P, P, P]
    L.gca_lin_blocks.argtypes = [P, P, P, P, P, I32, P, P, P, I32, I64, I32, I32, I32, P, P, P]
    L.gca_coll_blocks.argtypes = [P, P, P, P, P, P, I32, P, P, P, I32, I64, I32, I32, I32, P, P, P]
    L.gca_curved_entries.argtypes = [P, P, I64, P, P, I64, I32, I32, I32, I32, I32, P, P]
    L.gca_lin_build.argtypes = [P, I32, P, P, P]
    L.gca_lin_matvec.argtypes = [P, P, P, P]
    L.gca_lin_info.argtypes = [P, P]
    L.gca_lin_export.argtypes = [P, P, P, P]
    L.gca_lin_destroy.argtypes = [P]
    L.gca_lin_destroy.restype = None
    L.gca_destroy.argtypes = [P]
    L.gca_destroy.restype = None
    L.gca_last_error.argtypes = []
    L.gca_last_error.restype = ctypes.c_char_p
    for name in ("gca_tree_build", "gca_tree_info", "gca_tree_export", "gca_block_tree", "gca_build",
                 "h2_matvec",
                 "gca_entries", "gca_basis_sizes", "gca_basis_export", "gca_stats", "gca_phase_times",
                 "gca_solve_refined", "gca_update_geometry", "h2_bilinear_grad", "gca_store_blocks", "gca_energy", "gca_energy_noalloc",
                 "gca_block_entries", "gca_dl_entries", "gca_lin_vertex_triangles", "gca_lin_merge", "gca_lin_blocks",
                 "gca_coll_blocks", "gca_curved_entries", "gca_lin_build", "gca_lin_matvec", "gca_lin_info",
                 "gca_lin_export"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(code):
    if code != 0:
        raise Error(code, lib().gca_last_error().decode())


@dataclass
class Params:
    eta: float = 2.0
    eps: float = 1e-6
    omega_scale: float = 0.25
    green_m: int = 3
    q_A: int = 3
    q_r: int = 3
    q_nr: int = 3
    q_s: int = 4
    q_c: int = 3
    sym_rules: int = 0   # 1: symmetric triangle rules (3 / 6 points) for the disjoint pairs
    ss_fp32: int = 0     # 1: FP32 Gauss loops of the Sauter-Schwab rules in the mixed product
    serial: int = 0      # 1: every phase of a product on the caller's stream in order
    allocator: str = "torch"   # "torch": torch's caching allocator; None: hipMalloc / hipFree

    def _c(self):
        p = _Params()
        p.eta, p.eps, p.omega_scale = self.eta, self.eps, self.omega_scale
        p.green_m, p.q_A, p.q_r, p.q_nr, p.q_s = self.green_m, self.q_A, self.q_r, self.q_nr, self.q_s
        p.q_c = self.q_c
        p.sym_rules = self.sym_rules
        p.ss_fp32 = self.ss_fp32
        p.serial = self.serial
        if self.allocator == "torch":
            p.alloc, p.free = _TORCH_ALLOC, _TORCH_FREE
        elif self.allocator is not None:
            raise ValueError("allocator must be 'torch' or None")
        return p


class _MeshArrays:
    def __init__(self, verts, tris):
        self.xyz = np.ascontiguousarray(verts, dtype=np.float64)
        self.tri = np.ascontiguousarray(tris, dtype=np.int32)
        self.c = _Mesh(self.xyz.shape[0], self.tri.shape[0], self.xyz.ctypes.data, self.tri.ctypes.data)


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Tree:
    """Cluster tree (gca_tree_build); host only."""

    def __init__(self, verts, tris, leaf=64):
        self._m = _MeshArrays(verts, tris)
        self.h = ctypes.c_void_p()
        _check(lib().gca_tree_build(ctypes.byref(self._m.c), int(leaf), ctypes.byref(self.h)))

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().gca_tree_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def export(self):
        nc, depth = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().gca_tree_info(self.h, ctypes.byref(nc), ctypes.byref(depth)))
        perm = np.zeros(self._m.tri.shape[0], dtype=np.int32)
        nodes = np.zeros((nc.value, 5), dtype=np.int32)
        boxes = np.zeros((nc.value, 7))
        _check(lib().gca_tree_export(self.h, perm.ctypes.data, nodes.ctypes.data, boxes.ctypes.data))
        return perm, nodes, boxes


    def blocks(self, eta):
        """Admissible (t < s) and inadmissible leaf (t <= s) blocks as (k, 2) arrays."""
        nf, nn = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().gca_block_tree(self.h, float(eta), 0, None, ctypes.byref(nf), 0, None, ctypes.byref(nn)))
        far = np.zeros(2 * max(nf.value, 1), dtype=np.int32)
        near = np.zeros(2 * max(nn.value, 1), dtype=np.int32)
        _check(lib().gca_block_tree(self.h, float(eta), nf.value, far.ctypes.data, ctypes.byref(nf),
                                    nn.value, near.ctypes.data, ctypes.byref(nn)))
        far = np.stack([far[:nf.value], far[nf.value:2 * nf.value]], axis=1)
        near = np.stack([near[:nn.value], near[nn.value:2 * nn.value]], axis=1)
        return far, near


_live = weakref.WeakSet()


@atexit.register
def _close_live_handles():
    # handles whose memory came from torch's allocator go back to it while
    # torch is still alive
    for H in list(_live):
        try:
            H.close()
        except Exception:
            pass


class LinH2:
    """GCA-H^2 approximation of the nodal-basis matrix (gca_lin_build): one
    basis function per vertex; q_r / q_c / q_s / sym_rules of `params` are
    the rules of the stored nearfield and coupling blocks."""

    INFO = ("n", "clusters", "far_blocks", "near_blocks", "max_rank", "sum_rank", "far_entries", "near_entries")

    def __init__(self, verts, tris, leaf=16, params: Params = None, stream=None):
        self._m = _MeshArrays(verts, tris)
        self.params = params or Params()
        self.n = self._m.xyz.shape[0]
        self.h = ctypes.c_void_p()
        p = self.params._c()
        _check(lib().gca_lin_build(ctypes.byref(self._m.c), int(leaf), ctypes.byref(p), _stream_ptr(stream),
                                   ctypes.byref(self.h)))
        _live.add(self)

    def close(self):
        if getattr(self, "h", None):
            lib().gca_lin_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def matvec(self, x, stream=None):
        """y = G~ x (FP64 cuda tensors of n_v entries, original vertex order)."""
        import torch
        assert x.dtype == torch.float64 and x.is_cuda and x.dim() == 1 and x.shape[0] == self.n
        x = x.contiguous()
        y = torch.empty_like(x)
        _check(lib().gca_lin_matvec(self.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                    _stream_ptr(stream)))
        return y

    def info(self):
        a = np.zeros(8, dtype=np.int64)
        _check(lib().gca_lin_info(self.h, a.ctypes.data))
        return dict(zip(self.INFO, (int(v) for v in a)))

    def export(self):
        """(perm, ranks, pivots per cluster as a list of vertex-id arrays)."""
        inf = self.info()
        perm = np.zeros(self.n, dtype=np.int32)
        ranks = np.zeros(inf["clusters"], dtype=np.int32)
        piv = np.zeros(max(inf["sum_rank"], 1), dtype=np.int32)
        _check(lib().gca_lin_export(self.h, perm.ctypes.data, ranks.ctypes.data, piv.ctypes.data))
        off = np.concatenate([[0], np.cumsum(ranks)])
        return perm, ranks, [piv[off[c]:off[c + 1]] for c in range(len(ranks))]


class H2:
    """GCA-H^2 approximation (gca_build) on the current HIP device."""

    def __init__(self, verts, tris, tree: Tree, params: Params = None, stream=None):
        self._m = _MeshArrays(verts, tris)
        self.params = params or Params()
        self.n = self._m.tri.shape[0]
        self.h = ctypes.c_void_p()
        p = self.params._c()
        _check(lib().gca_build(ctypes.byref(self._m.c), tree.h, ctypes.byref(p), _stream_ptr(stream),
                               ctypes.byref(self.h)))
        _live.add(self)

    def close(self):
        if getattr(self, "h", None):
            lib().gca_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def matvec_into(self, x, y, precision=FP64, stream=None):
        """y = G~ x for torch cuda tensors (n,) or (n, nrhs) column-major
        (x.T contiguous), both float64 or both float32; raw call of h2_matvec."""
        import torch
        assert x.dtype == y.dtype and x.dtype in (torch.float64, torch.float32) and x.is_cuda and y.is_cuda
        if x.dim() == 1:
            nrhs, ld = 1, x.shape[0]
        else:
            nrhs, ld = x.shape[1], x.stride(1)
            assert x.stride(0) == 1 and y.stride(0) == 1 and y.stride(1) == ld
        dt = F32 if x.dtype == torch.float32 else F64
        _check(lib().h2_matvec(self.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                               nrhs, ld, dt, int(precision), _stream_ptr(stream)))
        return y

    def matvec(self, x, precision=FP64, stream=None):
        import torch
        if x.dim() == 1:
            xx = x.contiguous()
            y = torch.empty_like(xx)
        else:
            xx = x.t().contiguous().t()
            y = torch.empty_like(xx.t()).t()
        return self.matvec_into(xx, y, precision, stream)

    def energy(self, u, precision=FP64, scale=None, want_e=True, want_g=False, stream=None):
        """gca_energy: (E, g) with E = 1/2 u^T G~ u (0-dim tensor) and
        g = scale * G~ u (scale: 0-dim device tensor or None for 1); either
        may be skipped (None returned)."""
        import torch
        u = u.contiguous()
        assert u.dtype == torch.float64 and u.is_cuda and u.shape == (self.n,)
        e = torch.empty((), dtype=torch.float64, device=u.device) if want_e else None
        g = torch.empty_like(u) if want_g else None
        sc = None
        if scale is not None:
            sc = scale.detach().to(dtype=torch.float64).contiguous()
            assert sc.is_cuda and sc.numel() == 1
        _check(lib().gca_energy(self.h, _vp(u), _vp(sc) if sc is not None else None,
                                _vp(e) if e is not None else None, _vp(g) if g is not None else None,
                                int(precision), _stream_ptr(stream)))
        return e, g

    def energy_noalloc(self, u, precision=FP64, scale=None, want_e=True, want_g=False, stream=None):
        """gca_energy_noalloc: as energy(), with the library's fixed device
        workspace instead of allocated memory (the result tensors are the
        caller's, allocated here before the call)."""
        import torch
        u = u.contiguous()
        assert u.dtype == torch.float64 and u.is_cuda and u.shape == (self.n,)
        e = torch.empty((), dtype=torch.float64, device=u.device) if want_e else None
        g = torch.empty_like(u) if want_g else None
        sc = None
        if scale is not None:
            sc = scale.detach().to(dtype=torch.float64).contiguous()
            assert sc.is_cuda and sc.numel() == 1
        _check(lib().gca_energy_noalloc(self.h, _vp(u), _vp(sc) if sc is not None else None,
                                        _vp(e) if e is not None else None, _vp(g) if g is not None else None,
                                        int(precision), _stream_ptr(stream)))
        return e, g

    def solve(self, f, rtol=1e-8, max_outer=20, inner_rtol=1e-3, max_inner=500, stream=None):
        """u with ||f - G~ u|| <= rtol ||f|| (mixed CG inside FP64 refinement).
        Returns (u, outer steps, inner iterations, relative residual)."""
        import torch
        f = f.contiguous()
        assert f.dtype == torch.float64 and f.is_cuda and f.shape == (self.n,)
        u = torch.empty_like(f)
        it = (ctypes.c_int32 * 2)()
        rel = ctypes.c_double()
        _check(lib().gca_solve_refined(self.h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                       float(rtol), int(max_outer), float(inner_rtol), int(max_inner), it,
                                       ctypes.byref(rel), _stream_ptr(stream)))
        return u, it[0], it[1], rel.value

    def store_blocks(self, fp64=True, mixed=True, stream=None):
        """Compute the coupling and nearfield block rows once and keep them
        (gca_store_blocks); products in a stored precision read them.
        store_blocks(False, False) releases the storage."""
        which = (1 << FP64 if fp64 else 0) | (1 << MIXED if mixed else 0)
        _check(lib().gca_store_blocks(self.h, which, _stream_ptr(stream)))

    def dl_entries(self, I, J, stream=None):
        """gca_dl_entries: double-layer entries k_ij for the pairs (I[k], J[k])
        (original triangle ids), FP64, as a CUDA tensor."""
        import torch
        I = torch.as_tensor(np.ascontiguousarray(I), dtype=torch.int32).cuda()
        J = torch.as_tensor(np.ascontiguousarray(J), dtype=torch.int32).cuda()
        out = torch.empty(I.numel(), dtype=torch.float64, device="cuda")
        _check(lib().gca_dl_entries(self.h, _vp(I), _vp(J), I.numel(), _vp(out), _stream_ptr(stream)))
        return out

    def block_entries(self, precision=FP64, kind=0, stream=None):
        """gca_block_entries: (rows, cols, vals) of the stored coupling
        (kind 0) or nearfield (kind 1) block entries of one precision, with
        original triangle ids (numpy arrays; store_blocks first)."""
        L = lib()
        cnt = ctypes.c_int64(0)
        _check(L.gca_block_entries(self.h, int(precision), int(kind), 0, None, None, None, ctypes.byref(cnt),
                                   _stream_ptr(stream)))
        k = cnt.value
        r = np.empty(k, dtype=np.int32)
        c = np.empty(k, dtype=np.int32)
        v = np.empty(k, dtype=np.float64)
        _check(L.gca_block_entries(self.h, int(precision), int(kind), k, r.ctypes.data, c.ctypes.data,
                                   v.ctypes.data, None, _stream_ptr(stream)))
        return r, c, v

    def update_geometry(self, verts, stream=None):
        """Move the vertices keeping tree, blocks, boxes, Green points and pivots
        (frozen structure); bases are recomputed from the Green factor."""
        v = np.ascontiguousarray(verts, dtype=np.float64)
        assert v.shape == self._m.xyz.shape
        _check(lib().gca_update_geometry(self.h, v.ctypes.data, _stream_ptr(stream)))

    def bilinear_grad(self, a, b, alpha=1.0, dxyz=None, precision=FP64, scale=None, stream=None):
        """dxyz += alpha * scale * d(a^T G~ b)/dX (frozen structure; scale: 0-dim
        device tensor or None for 1); returns dxyz (nv, 3)."""
        import torch
        a = a.contiguous()
        b = b.contiguous()
        if dxyz is None:
            dxyz = torch.zeros((self._m.xyz.shape[0], 3), dtype=torch.float64, device=a.device)
        sc = None
        if scale is not None:
            sc = scale.detach().to(dtype=torch.float64).contiguous()
            assert sc.is_cuda and sc.numel() == 1
        _check(lib().h2_bilinear_grad(self.h, ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                      float(alpha), _vp(sc) if sc is not None else None,
                                      ctypes.c_void_p(dxyz.data_ptr()), int(precision), _stream_ptr(stream)))
        return dxyz

    def entries(self, I, J, precision=FP64, stream=None):
        import torch
        I = torch.as_tensor(I, dtype=torch.int32).cuda().contiguous()
        J = torch.as_tensor(J, dtype=torch.int32).cuda().contiguous()
        out = torch.empty(I.shape[0], dtype=torch.float64, device=I.device)
        _check(lib().gca_entries(self.h, ctypes.c_void_p(I.data_ptr()), ctypes.c_void_p(J.data_ptr()),
                                 I.shape[0], ctypes.c_void_p(out.data_ptr()), int(precision),
                                 _stream_ptr(stream)))
        return out

    def basis(self):
        """ranks per cluster, pivots (original ids, per cluster in pivot order),
        leaf V and transfer E entries (flat, see include/gca.h)."""
        npv, nb = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().gca_basis_sizes(self.h, ctypes.byref(npv), ctypes.byref(nb)))
        st = self.stats()
        ranks = np.zeros(st["n_clusters"], dtype=np.int32)
        piv = np.zeros(npv.value, dtype=np.int32)
        basis = np.zeros(nb.value)
        _check(lib().gca_basis_export(self.h, ranks.ctypes.data, piv.ctypes.data, basis.ctypes.data))
        return ranks, piv, basis

    def stats(self):
        s = _Stats()
        _check(lib().gca_stats(self.h, ctypes.byref(s)))
        out = {k: getattr(s, k) for k, _ in _Stats._fields_ if k not in ("phase_ms", "setup_ms", "reserved_i")}
        out["setup_ms"] = dict(zip(["mesh_adjacency", "pair_lists", "block_tree", "geometry", "basis",
                                    "slots_lists"], list(s.setup_ms)[:6]))
        out["phase_ms"] = dict(zip(PHASES, list(s.phase_ms)))
        return out

    def phase_times(self, max_products=64):
        """Per-product phase times (ms) of the last products, shape (count, 10)."""
        cnt = ctypes.c_int64()
        _check(lib().gca_phase_times(self.h, int(max_products), None, ctypes.byref(cnt)))
        out = np.zeros((max(cnt.value, 1), len(PHASES)))
        _check(lib().gca_phase_times(self.h, int(max_products), out.ctypes.data, ctypes.byref(cnt)))
        return out[:cnt.value]


# ------------------------------------------------------------- autograd ----
# torch.autograd glue around h2_matvec and h2_bilinear_grad (marshalling only).
# The operator G~(X) is symmetric, so the vector-Jacobian product of
# y = G~ x with respect to x is G~ y_bar; with respect to the vertex
# coordinates X it is d(y_bar^T G~ x)/dX at frozen structure.  The vertex
# tensor passed in must hold the coordinates the operator was built or last
# updated at (H2.update_geometry); it only routes the gradient.

_autograd_fns = None


def _fns():
    global _autograd_fns
    if _autograd_fns is not None:
        return _autograd_fns
    import torch

    class _Matvec(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x, verts, H, precision):
            ctx.H, ctx.precision = H, precision
            ctx.save_for_backward(x)
            return H.matvec(x, precision)

        @staticmethod
        def backward(ctx, gy):
            (x,) = ctx.saved_tensors
            H, prec = ctx.H, ctx.precision
            gx = gv = None
            if ctx.needs_input_grad[0]:
                gx = H.matvec(gy, prec)
            if ctx.needs_input_grad[1]:
                gv = torch.zeros((H._m.xyz.shape[0], 3), dtype=torch.float64, device=x.device)
                if x.dim() == 1:
                    H.bilinear_grad(gy, x, 1.0, gv, prec)
                else:
                    for k in range(x.shape[1]):
                        H.bilinear_grad(gy[:, k], x[:, k], 1.0, gv, prec)
            return gx, gv, None, None

    class _Energy(torch.autograd.Function):
        @staticmethod
        def forward(ctx, u, verts, H, precision):
            ctx.H, ctx.precision = H, precision
            ctx.save_for_backward(u)
            e, _ = H.energy(u, precision)
            return e

        @staticmethod
        def backward(ctx, ge):
            (u,) = ctx.saved_tensors
            H, prec = ctx.H, ctx.precision
            du = dv = None
            if ctx.needs_input_grad[0]:
                _, du = H.energy(u, prec, scale=ge, want_e=False, want_g=True)
            if ctx.needs_input_grad[1]:
                dv = torch.zeros((H._m.xyz.shape[0], 3), dtype=torch.float64, device=u.device)
                H.bilinear_grad(u, u, 0.5, dv, prec, scale=ge)
            return du, dv, None, None

    _autograd_fns = (_Matvec, _Energy)
    return _autograd_fns


def matvec(H: "H2", x, verts=None, precision=FP64):
    """Differentiable y = G~ x: gradients flow to x and, if given, to the
    vertex tensor verts (nv x 3, float64, on x's device)."""
    import torch
    if verts is None:
        verts = torch.zeros((0,), dtype=torch.float64, device=x.device)
    return _fns()[0].apply(x, verts, H, precision)


def energy(H: "H2", u, verts=None, precision=FP64):
    """Differentiable E = 1/2 u^T G~ u (u: (n,) float64 cuda)."""
    import torch
    if verts is None:
        verts = torch.zeros((0,), dtype=torch.float64, device=u.device)
    return _fns()[1].apply(u, verts, H, precision)


# ---------------------------------------------------------------------------
# Continuous piecewise-linear nodal basis (Section 5)

LIN_MAX_GATHER, LIN_MAX_SET, LIN_MAX_BLOCK_SET, LIN_MAX_TRIS, LIN_MAX_DEGREE = 2048, 1024, 64, 192, 16


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


def lin_vertex_triangles(tris, nv):
    """The sets T_i (gca_lin_vertex_triangles, host): (off[nv + 1], list[3 nt])
    as int32 numpy arrays."""
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    nt = int(tris.shape[0])
    off = np.zeros(nv + 1, dtype=np.int32)
    lst = np.zeros(max(3 * nt, 1), dtype=np.int32)
    _check(lib().gca_lin_vertex_triangles(tris.ctypes.data_as(ctypes.c_void_p), nt, int(nv),
                                          off.ctypes.data_as(ctypes.c_void_p),
                                          lst.ctypes.data_as(ctypes.c_void_p)))
    return off, lst[:3 * nt]


def lin_merge(vt_off, vt_list, tri, set_off, set_vtx, cap, stream=None):
    """Merged triangle lists of vertex subsets (gca_lin_merge).  Inputs are
    int32 CUDA tensors; returns (tri[nsets, cap], loc[nsets, cap, 3],
    count[nsets]) as CUDA tensors (count -1 where a limit is exceeded)."""
    import torch
    nsets = int(set_off.numel()) - 1
    dev = set_off.device
    out_tri = torch.full((max(nsets, 1), cap), -1, dtype=torch.int32, device=dev)
    out_loc = torch.full((max(nsets, 1), cap, 3), -1, dtype=torch.int32, device=dev)
    out_count = torch.zeros(max(nsets, 1), dtype=torch.int32, device=dev)
    _check(lib().gca_lin_merge(_vp(vt_off), _vp(vt_list), _vp(tri), _vp(set_off), _vp(set_vtx), nsets, int(cap),
                               _vp(out_tri), _vp(out_loc), _vp(out_count), _stream_ptr(stream)))
    return out_tri[:nsets], out_loc[:nsets], out_count[:nsets]


def lin_blocks(xyz, tri, merged, set_off, blk_row, blk_col, ld, q, sym=False, q_s=0, stream=None):
    """Dense FP64 linear-basis blocks (gca_lin_blocks) over the merged lists
    `merged` = (tri, loc, count) of lin_merge; q_s > 0 integrates touching
    pairs by the Sauter-Schwab rules.  Returns (out[nblk, ld], status[nblk])
    as CUDA tensors."""
    import torch
    m_tri, m_loc, m_count = merged
    cap = int(m_tri.shape[1])
    nblk = int(blk_row.numel())
    out = torch.empty((max(nblk, 1), ld), dtype=torch.float64, device=xyz.device)
    status = torch.empty(max(nblk, 1), dtype=torch.int32, device=xyz.device)
    _check(lib().gca_lin_blocks(_vp(xyz), _vp(tri), _vp(m_tri), _vp(m_loc), _vp(m_count), cap, _vp(set_off),
                                _vp(blk_row), _vp(blk_col), nblk, int(ld), int(q), int(bool(sym)), int(q_s),
                                _vp(out), _vp(status), _stream_ptr(stream)))
    return out[:nblk], status[:nblk]


def coll_blocks(xyz, tri, set_vtx, merged, set_off, blk_row, blk_col, ld, q, sym=False, q_s=8, stream=None):
    """Dense FP64 collocation blocks of the linear nodal basis (gca_coll_blocks):
    rows the vertices of the row subsets (collocation points), columns the
    nodal functions of the column subsets over their merged lists `merged`
    = (tri, loc, count) of lin_merge.  Returns (out[nblk, ld], status[nblk])
    as CUDA tensors."""
    import torch
    m_tri, m_loc, m_count = merged
    cap = int(m_tri.shape[1])
    nblk = int(blk_row.numel())
    out = torch.empty((max(nblk, 1), ld), dtype=torch.float64, device=xyz.device)
    status = torch.empty(max(nblk, 1), dtype=torch.int32, device=xyz.device)
    _check(lib().gca_coll_blocks(_vp(xyz), _vp(tri), _vp(set_vtx), _vp(m_tri), _vp(m_loc), _vp(m_count), cap,
                                 _vp(set_off), _vp(blk_row), _vp(blk_col), nblk, int(ld), int(q), int(bool(sym)),
                                 int(q_s), _vp(out), _vp(status), _stream_ptr(stream)))
    return out[:nblk], status[:nblk]


def curved_entries(nodes, tri6, I, J, op=0, basis=0, q=3, sym=False, q_s=4, stream=None):
    """Galerkin moments of curved (quadratic) triangle pairs (gca_curved_entries):
    nodes (nn, 3) FP64 and tri6 (nt, 6) int32 CUDA tensors, I and J int32 CUDA
    tensors of triangle ids; op 0 single layer, 1 double layer; basis 0 the
    piecewise-constant entries (m,), basis 1 the nine nodal moments (m, 3, 3).
    Returns a CUDA FP64 tensor."""
    import torch
    m = int(I.numel())
    assert int(J.numel()) == m and I.dtype == torch.int32 and J.dtype == torch.int32
    assert nodes.dtype == torch.float64 and tri6.dtype == torch.int32 and tri6.shape[1] == 6
    assert nodes.is_contiguous() and tri6.is_contiguous() and I.is_contiguous() and J.is_contiguous()
    out = torch.empty(max(m, 1) * (9 if basis else 1), dtype=torch.float64, device=nodes.device)
    _check(lib().gca_curved_entries(_vp(nodes), _vp(tri6), int(tri6.shape[0]), _vp(I), _vp(J), m, int(op),
                                    int(basis), int(q), int(bool(sym)), int(q_s), _vp(out), _stream_ptr(stream)))
    return out[:m * 9].view(m, 3, 3) if basis else out[:m]
