#!/usr/bin/env python3
"""Throughput of the GCA-H^2 matrix-vector product on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload sphere_l8]

One step = one H^2 product y = G~ x (forward transform, coupling blocks and
nearfield blocks recomputed by pair quadrature, backward transform, touching
pairs) for one right-hand side, inputs resident in HBM.  `value` is
DoF/s = n / (seconds per product) of the mixed-precision path (FP32
regular-pair quadrature and transfers, FP64 Sauter-Schwab touching pairs); the
FP64 path is measured on the same H^2 approximation alongside, and so is the
opt-in variant with FP32 Sauter-Schwab Gauss loops (a second handle built with
ss_fp32 = 1).  Setup seconds cover tree
construction and gca_build (synchronised wall time).  The adjoint of the
energy with respect to the vertex coordinates is timed in both precisions
after the products (`energy_gradient`), and so is the stored-block mode
(`stored_blocks`: block rows computed once, products read them).  The
piecewise-linear nodal basis (`linear_basis`) is measured on the same mesh:
the merge of vertex-subset triangle lists and FP64 Galerkin blocks assembled
triangle pair by triangle pair, against its own FP64 ceiling.  The refined
solve of G u = f (mixed CG inside FP64 refinement to 1e-8) is timed on the
level-7 sphere (`solve_level7`).

The roofline object describes the dominant kernel of the mixed product, timed
with the library's per-product HIP events over the timed steps: `frac` is
against the published FP32 vector peak (157.3 TFLOP/s, 10 flops per kernel
evaluation), `issue_ceiling_frac` against the instruction-mix ceiling of an
evaluation (5 full-rate VALU lane-ops and one quarter-rate rsqrt).  The CPU
baseline is the plain FP64 oracle computing sampled rows of G x on the host
cores; the same rows give the relative error of both GPU paths for three
vectors (x ~ N(0,1), the all-ones vector and the centroid x3 coordinates), and
the reported error is the largest of the three.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "H² matvec DoF/s + setup s at 1e-4 rel err: mixed vs FP64 plain, % roofline"

# ALU ceiling of one FP32 kernel evaluation w / |x - y| accumulated into a sum
# with the squared distance expanded around
# reference points, 5 VALU lane-ops (1 add + 3 fma for |x - y|^2, 1 fma to
# accumulate) + 1 v_rsq_f32.  The published FP32 vector peak, 157.3 TFLOP/s =
# 256 CUs x 2.4 GHz x 128 FMA lanes per clock, gives 7.86e13 lane-ops/s;
# transcendentals run at a quarter of that.  Algorithmic work is counted as 10
# flops per evaluation.
VALU_LANE_OPS_PER_S = 256 * 128 * 2.4e9
TRANS_LANE_OPS_PER_S = VALU_LANE_OPS_PER_S / 4
FLOPS_PER_EVAL = 10
GRAD_FLOPS_PER_EVAL = 18
EVALS_PER_S_F32 = 1.0 / (5.0 / VALU_LANE_OPS_PER_S + 1.0 / TRANS_LANE_OPS_PER_S)
ISSUE_CEILING_F32_TFLOPS = EVALS_PER_S_F32 * FLOPS_PER_EVAL / 1e12
# the published FP32 vector peak of the chip (packed FP32 FMA: 256 CUs x
# 2.4 GHz x 128 lanes x 2 flops)
PUBLISHED_F32_TFLOPS = 157.3
PUBLISHED_F64_TFLOPS = 78.6     # FP64 vector and FP64 matrix peak


# FP64 ceiling of one dimension-reduced Sauter-Schwab evaluation (the
# touching kernels): about 12 FP64 VALU operations (point difference,
# squared norm, rsqrt refinement, weighted accumulate) and one FP64 rsqrt at
# a quarter of the VALU rate.  FP64 vector peak 78.6 TFLOP/s = 3.93e13
# FMA lane-ops/s.
FP64_LANE_OPS_PER_S = 78.6e12 / 2
SS_EVALS_PER_S = 1.0 / (12.0 / FP64_LANE_OPS_PER_S + 1.0 / (FP64_LANE_OPS_PER_S / 4))
HBM_BYTES_PER_S = 8.0e12
# The mixed product's touching kernels run their Gauss loops in FP32: about
# 10 FP32 VALU lane-ops per dimension-reduced point (point, squared norm,
# weighted accumulate) and one quarter-rate v_rsq_f32.
SS_EVALS_PER_S_F32 = 1.0 / (10.0 / VALU_LANE_OPS_PER_S + 1.0 / TRANS_LANE_OPS_PER_S)


# FP64 ceiling of the linear-basis block kernel per kernel evaluation: 3 FP64
# subtractions, 3 for |x - y|^2, 4 for the refined rsqrt and its quarter-rate
# v_rsq_f64 (4 issue slots), 3 FMAs for the three column-corner moments, and
# the 27 FMAs that fold the P column sums into the nine corner moments of the
# pair, shared by its P evaluations of one row point.
def lin_evals_per_s(P):
    return FP64_LANE_OPS_PER_S / (13.0 + 4.0 + 27.0 / P)


# FP64 ceiling of one collocation evaluation (a rule point of a column
# triangle against a collocation point): 6 FMAs for the point, 3 subtractions,
# 3 operations for |x - y|^2, 4 for the refined rsqrt plus the quarter-rate
# v_rsq_f64 (4 issue slots), 1 FMA for the weighted sum: 17 + 4 slots.
COLL_EVALS_PER_S = FP64_LANE_OPS_PER_S / 21.0


# FP64 ceilings of the curved-triangle kernels (quadratic maps, normals
# interpolated from their six nodal values).  Regular pairs: per kernel
# evaluation 3 subtractions, 3 for |x - y|^2, the refined rsqrt (4 slots)
# with its quarter-rate v_rsq_f64 (4), the Gramian factor and the weighted
# sum (2): 16 slots; per rule point (2 P per pair) the shape functions (11),
# the point and the normal (33 FMAs), |n|^2 and the square root (about 11):
# 55 slots.  Touching pairs, per 4D point: the map and its weight (12), two
# points with their normals (88), the differences, norms, refined rsqrt and
# weight (25), the sum (1): 126 slots.
def curved_pairs_per_s(P):
    return FP64_LANE_OPS_PER_S / (16.0 * P * P + 55.0 * 2 * P)


CURVED_SS_EVALS_PER_S = FP64_LANE_OPS_PER_S / 126.0


def phase_rooflines(st, params, P, Pc, ms, ss_fp32=False):
    """Fraction of its bound for every phase of the mixed product (per
    product): the quadrature phases against the FP32 ALU ceiling (10 flops
    per evaluation), the touching lists against the FP32 evaluation ceiling,
    the transforms and the gather against HBM with their algorithmic bytes
    (FP32 basis entries read once, vectors read or written once)."""
    q = params.q_s
    nv_, ne_ = st["basis_entries_leaf"], st["basis_entries_transfer"]
    n = st["n"]
    out = {}
    for ph, flops in (("near_blocks", st["near_regular_pairs"] * P * P * FLOPS_PER_EVAL),
                      ("coupling_blocks", st["coupling_entries"] * Pc * Pc * FLOPS_PER_EVAL)):
        a = flops / (ms[ph] * 1e-3) / 1e12
        out[ph] = {"bound": "alu", "achieved": a, "peak": PUBLISHED_F32_TFLOPS, "unit": "TFLOP/s",
                   "frac": a / PUBLISHED_F32_TFLOPS, "issue_ceiling": ISSUE_CEILING_F32_TFLOPS,
                   "issue_ceiling_frac": a / ISSUE_CEILING_F32_TFLOPS}
    ev = st["n_ident"] * 3 * q + st["n_edge"] * 5 * q * q + st["n_vert"] * 2 * q ** 3
    a = ev / (ms["touching"] * 1e-3)
    peak = SS_EVALS_PER_S_F32 if ss_fp32 else SS_EVALS_PER_S
    out["touching"] = {"bound": "alu", "achieved": a, "peak": peak, "unit": "evaluations/s",
                       "frac": a / peak, "arithmetic": "FP32 Gauss loops" if ss_fp32 else "FP64"}
    for ph, byts in (("forward", 4 * (nv_ + ne_) + 4 * n),
                     ("backward", 4 * ne_),
                     ("gather", 4 * nv_ + 2 * (st["n_edge"] + st["n_vert"]) * 12 + st["n_ident"] * 12 + 8 * n)):
        a = byts / (ms[ph] * 1e-3)
        out[ph] = {"bound": "hbm", "achieved": a / 1e9, "peak": HBM_BYTES_PER_S / 1e9, "unit": "GB/s",
                   "frac": a / HBM_BYTES_PER_S, "bytes": byts}
    return out


def rule_points(q, sym):
    """Points per triangle of the rule of order q: q^2 (collapsed Gauss) or
    the symmetric rule of the same degree (3 points for q = 2, 6 for q = 3)."""
    return {2: 3, 3: 6}[q] if sym else q * q


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed PMC summary
    (profiles/pmc_traffic_sphere_l8.md), or None when the kernel's source has
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic_sphere_l8.md")
    src = os.path.join(ROOT, "paper_1810_08429_amd", "csrc", "quad.hip")
    try:
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
        for line in open(path):
            f = line.split()
            if line.startswith("machine-readable: traffic_bytes") and f[2] == kernel and f[-1] == digest:
                return float(f[3])
    except OSError:
        pass
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sphere_l8")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target wall time of the oracle CPU baseline sample (0 disables it)")
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--err-rows", type=int, default=384,
                    help="rows of the oracle accuracy sample (fewer if they do not fit the CPU budget)")
    ap.add_argument("--eps", type=float, default=None, help="override the workload's ACA tolerance")
    ap.add_argument("--q-nr", type=int, default=None, help="override the near-regular pair order")
    ap.add_argument("--q-c", type=int, default=None, help="override the coupling-entry rule order")
    ap.add_argument("--sym", type=int, default=None, choices=(0, 1),
                    help="override the workload's triangle-rule family for disjoint pairs "
                         "(0 collapsed Gauss, 1 symmetric)")
    ap.add_argument("--stored-steps", type=int, default=10,
                    help="timed products per precision in stored-block mode (0 disables it)")
    ap.add_argument("--grad-steps", type=int, default=3,
                    help="timed calls of the energy gradient per precision (0 disables it)")
    ap.add_argument("--solve-steps", type=int, default=1,
                    help="timed refined solves on the level-7 sphere (0: skip)")
    ap.add_argument("--nodal-level", type=int, default=7,
                    help="sphere level of the nodal-basis H2 timing leg (0: skip)")
    ap.add_argument("--lin-blocks", type=int, default=16384,
                    help="linear-basis blocks (32 x 32 vertices) in the piecewise-linear leg (0 disables it)")
    ap.add_argument("--omega", type=float, default=None, help="override the workload's omega margin")
    ap.add_argument("--green-m", type=int, default=None, help="override the workload's Green order")
    ap.add_argument("--ss32-steps", type=int, default=10,
                    help="timed mixed products of a handle built with FP32 Sauter-Schwab loops (0 disables it)")
    ap.add_argument("--serial-steps", type=int, default=10,
                    help="timed mixed products of a handle built with serial = 1 (every phase alone on the "
                         "caller's stream: per-kernel rooflines in isolation; 0 disables it)")
    ap.add_argument("--rhs16-steps", type=int, default=5,
                    help="timed batched products with 16 right-hand sides per precision (0 disables it)")
    ap.add_argument("--curved-rows", type=int, default=32768,
                    help="random triangles whose touching pairs the curved-triangle leg integrates (0: skip)")
    ap.add_argument("--dl-rows", type=int, default=32768,
                    help="triangles whose touching pairs (and as many random pairs) time the double-layer entries "
                         "(0 disables it)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 1 GiB device copy (calibrates the PMC byte counters)")
    return ap.parse_args()


def solve_leg(gca, torch, steps):
    """The level-7 sphere (327,680 triangles) with the settings of the
    level-8 operating point (leaf 64, eta 2, Green order 5, omega margin 1.5,
    eps 1e-5, coupling order 2, symmetric rules): G u = f with
    f_i = int_{t_i} x_3 solved by CG on the mixed product inside FP64
    refinement to a relative residual of 1e-8 (gca_solve_refined).  Setup and
    solve wall times, the iteration counts, and the L2 distance of u to the
    exact density 3 x_3 of the unit sphere (the best piecewise-constant
    approximation is itself O(h) away)."""
    import synth
    m = synth.icosphere(7)
    _, prm = synth.workload("sphere_l8")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p = gca.Params(eta=prm["eta"], eps=prm["eps"], green_m=prm["green_m"], omega_scale=prm["omega_scale"])
    p.q_c = prm["q_c"]
    p.sym_rules = prm["sym_rules"]
    H = gca.H2(m.verts, m.tris, gca.Tree(m.verts, m.tris, prm["leaf"]), p)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    T = m.verts[m.tris]
    area = 0.5 * np.linalg.norm(np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0]), axis=1)
    c = T.mean(axis=1)
    f = torch.tensor(area * c[:, 2], device="cuda")
    H.solve(f, rtol=1e-8, max_inner=2000)   # untimed: the solver's workspaces
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        u, outer, inner, rel = H.solve(f, rtol=1e-8, max_inner=2000)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / steps
    uu = u.cpu().numpy()
    exact = 3.0 * c[:, 2]
    err = float(np.sqrt(np.sum(area * (uu - exact) ** 2) / np.sum(area * exact ** 2)))
    H.close()
    res = {"workload": "unit icosphere level 7, 327680 flat triangles, the level-8 operating point's settings "
                       "(leaf 64, eta 2, Green order 5, omega margin 1.5, ACA eps 1e-5, coupling order 2, symmetric "
                       "rules); f_i = int_{t_i} x_3; mixed-precision CG inside FP64 refinement to 1e-8",
           "n": int(m.nt), "setup_s": t_setup, "solve_ms": dt * 1e3, "steps": steps, "outer": int(outer),
           "inner": int(inner), "relres": float(rel), "density_rel_err_l2": err}
    print(f"[bench] solve level 7 (n = {m.nt}): setup {t_setup:.2f} s, solve {dt * 1e3:.1f} ms "
          f"({outer} refinement steps, {inner} CG iterations, residual {rel:.1e}), |u - 3 x3| {err:.2e}",
          file=sys.stderr, flush=True)
    return res


def lin_h2(gca, torch, level_time, level_err=5, steps=10, leaf=32):
    """GCA-H^2 with the nodal basis (gca_lin_build / gca_lin_matvec): the
    approximation error of the product at level `level_err` against the same
    handle built with eta -> 0 (every block stored as nearfield: the nodal
    Galerkin matrix itself), for x ~ N(0,1), the all-ones vector and x3; then
    build time, storage and the product time (HIP events) at level
    `level_time`."""
    import synth
    prm = dict(eta=2.0, eps=1e-5, omega_scale=0.25, green_m=4, q_A=2, q_r=3, q_nr=3, q_s=4, q_c=2, sym_rules=1)
    res = {"workload": f"unit icosphere, nodal basis (one function per vertex), leaf {leaf}, eta 2, Green order 4, "
                       f"ACA eps 1e-5, Green factor rule q_A 2, symmetric 6-point rule for the nearfield pairs and "
                       f"3-point rule for the coupling entries, Sauter-Schwab q_s 4 for touching pairs; FP64",
           "params": prm}
    m = synth.icosphere(level_err)
    P = gca.Params(**prm)
    H = gca.LinH2(m.verts, m.tris, leaf=leaf, params=P)
    D = gca.LinH2(m.verts, m.tris, leaf=leaf, params=gca.Params(**{**prm, "eta": 1e-9}))
    X = error_vectors_nodal(m, synth.rhs_normal(m.nv, seed=0))
    errs = {}
    for k, name in enumerate(("x_normal", "ones", "x3")):
        x = torch.as_tensor(np.ascontiguousarray(X[:, k])).cuda()
        y, yd = H.matvec(x), D.matvec(x)
        errs[name] = float((y - yd).abs().max() / yd.abs().max())
    res["error"] = {"level": level_err, "n": m.nv, "reference": "the same handle with eta -> 0 (all blocks stored "
                    "dense: the nodal Galerkin matrix with the same rules)", "max_rel": max(errs.values()),
                    "per_vector": errs, "info": H.info()}
    del D
    torch.cuda.empty_cache()
    m = synth.icosphere(level_time)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H = gca.LinH2(m.verts, m.tris, leaf=leaf, params=P)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    x = torch.as_tensor(synth.rhs_normal(m.nv, seed=0)).cuda()
    for _ in range(2):
        H.matvec(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        H.matvec(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    inf = H.info()
    # algorithmic bytes of a product: the stored entries once, the vectors and bases around them
    nbytes = 8 * (inf["far_entries"] + inf["near_entries"])
    res["time"] = {"level": level_time, "n": m.nv, "build_s": build_s, "ms_per_product": ms, "DoF_per_s": m.nv / (ms * 1e-3),
                   "info": inf, "stored_bytes": nbytes,
                   "roofline": {"bound": "hbm", "achieved": nbytes / (ms * 1e-3) / 1e9, "peak": HBM_BYTES_PER_S / 1e9,
                                "unit": "GB/s", "frac": nbytes / (ms * 1e-3) / HBM_BYTES_PER_S,
                                "what": "stored coupling and nearfield entries read once per product (FP64)"}}
    print(f"[bench] nodal H2: error {res['error']['max_rel']:.2e} at level {level_err}; level {level_time} "
          f"(n = {m.nv}): build {build_s:.2f} s, product {ms:.3f} ms, {nbytes / 1e9:.2f} GB stored, "
          f"{res['time']['roofline']['frac']:.1%} of HBM", file=sys.stderr, flush=True)
    return res


def error_vectors_nodal(mesh, x_host):
    """The error metric's vectors for the nodal basis: x ~ N(0,1), the all-ones
    vector and the vertex x3 coordinate."""
    return np.stack([x_host, np.ones(mesh.nv), mesh.verts[:, 2]], axis=1)


def linear_basis(gca, torch, mesh, nblk, steps, warmup, q=2, sym=True, seed=7):
    """Piecewise-linear nodal basis (Section 5) on the workload's mesh: nblk
    blocks, rows and columns each 32 vertices drawn at random from the 256
    nearest to a random centre (a stand-in for pivot sets of 32 vertices in a
    cluster), centres at least 0.1 apart.  Times the merge of all 2 nblk
    subsets and the block assembly with HIP events on the current stream."""
    from scipy.spatial import cKDTree
    import ctypes
    rng = np.random.default_rng(seed)
    c = rng.integers(mesh.nv, size=2 * nblk)
    while True:
        d = np.linalg.norm(mesh.verts[c[0::2]] - mesh.verts[c[1::2]], axis=1)
        bad = np.nonzero(d < 0.1)[0]
        if bad.size == 0:
            break
        c[2 * bad + 1] = rng.integers(mesh.nv, size=bad.size)
    _, nb = cKDTree(mesh.verts).query(mesh.verts[c], k=256)
    pick = np.argsort(rng.random(nb.shape), axis=1)[:, :32]
    sets = np.take_along_axis(nb, pick, axis=1).astype(np.int32)
    off, lst = gca.lin_vertex_triangles(mesh.tris, mesh.nv)
    cuda = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x), dtype=dt).cuda()
    xyz, tri = cuda(mesh.verts, torch.float64), cuda(mesh.tris, torch.int32)
    vt_off, vt_list = cuda(off, torch.int32), cuda(lst, torch.int32)
    set_off = cuda(np.arange(0, 32 * 2 * nblk + 1, 32), torch.int32)
    set_vtx = cuda(sets.reshape(-1), torch.int32)
    cap, ld, ns = 192, 32 * 32, 2 * nblk
    m_tri = torch.empty((ns, cap), dtype=torch.int32, device="cuda")
    m_loc = torch.empty((ns, cap, 3), dtype=torch.int32, device="cuda")
    m_cnt = torch.empty(ns, dtype=torch.int32, device="cuda")
    br = cuda(np.arange(0, ns, 2), torch.int32)
    bc = cuda(np.arange(1, ns, 2), torch.int32)
    out = torch.empty((nblk, ld), dtype=torch.float64, device="cuda")
    status = torch.empty(nblk, dtype=torch.int32, device="cuda")
    L = gca.lib()
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def merge():
        gca._check(L.gca_lin_merge(vp(vt_off), vp(vt_list), vp(tri), vp(set_off), vp(set_vtx), ns, cap,
                                   vp(m_tri), vp(m_loc), vp(m_cnt), sp))

    def blocks():
        gca._check(L.gca_lin_blocks(vp(xyz), vp(tri), vp(m_tri), vp(m_loc), vp(m_cnt), cap, vp(set_off), vp(br),
                                    vp(bc), nblk, ld, q, int(sym), 4, vp(out), vp(status), sp))

    def timed(fn):
        for _ in range(warmup):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    def coll():
        gca._check(L.gca_coll_blocks(vp(xyz), vp(tri), vp(set_vtx), vp(m_tri), vp(m_loc), vp(m_cnt), cap,
                                     vp(set_off), vp(br), vp(bc), nblk, ld, q, int(sym), 8, vp(out), vp(status),
                                     sp))

    merge_ms = timed(merge)
    blocks_ms = timed(blocks)
    coll_ms = timed(coll)
    cst = status.cpu().numpy()
    if (cst != 0).any():
        raise RuntimeError("collocation workload exceeded a kernel limit")
    # collocation evaluations: per row point, P per (triangle, local corner) of the column list
    # (the subsets of a block are at least 0.1 apart: no Duffy case)
    loc = m_loc.cpu().numpy()
    corners = np.array([(loc[k, :max(int(c), 0)] >= 0).sum() for k, c in
                        enumerate(m_cnt.cpu().numpy())], dtype=np.int64)
    cnt = m_cnt.cpu().numpy().astype(np.int64)
    st = status.cpu().numpy()
    if (cnt < 0).any() or (st != 0).any():
        raise RuntimeError("linear-basis workload exceeded a kernel limit or has touching blocks")
    P = rule_points(q, sym)
    evals = int((cnt[0::2] * cnt[1::2]).sum()) * P * P
    ach = evals / (blocks_ms * 1e-3)
    peak = lin_evals_per_s(P)
    res = {"workload": f"{nblk} blocks of 32 x 32 vertices on the workload mesh ({mesh.nv} vertices), each "
                       f"subset 32 of the 256 vertices nearest a random centre (seed {seed}), block centres >= 0.1 "
                       f"apart; regular rule {'symmetric' if sym else 'collapsed Gauss'} order {q} "
                       f"({P} points) on both triangles, FP64",
           "merge_ms": merge_ms, "subsets_per_s": ns / (merge_ms * 1e-3),
           "blocks_ms": blocks_ms, "entries_per_s": nblk * ld / (blocks_ms * 1e-3),
           "merged_rows_mean": float(cnt.mean()), "kernel_evaluations": evals,
           "roofline": {"bound": "fp64 alu", "achieved": ach, "peak": peak, "unit": "evaluations/s",
                        "frac": ach / peak, "kernel": f"k_lin_blocks<{P}>"},
           "steps": steps}
    cev = int(32 * corners[1::2].sum()) * P
    cach = cev / (coll_ms * 1e-3)
    res["collocation"] = {
        "what": "the collocation matrix of the same basis (Section 6): rows the 32 vertices of each block's row "
                "subset as collocation points, columns the nodal functions of its column subset, single integrals "
                "by the same regular rule (Duffy rule with 8 points where a point is a corner, absent here)",
        "blocks_ms": coll_ms, "entries_per_s": nblk * ld / (coll_ms * 1e-3), "kernel_evaluations": cev,
        "galerkin_over_collocation_time": blocks_ms / coll_ms,
        "roofline": {"bound": "fp64 alu", "achieved": cach, "peak": COLL_EVALS_PER_S, "unit": "evaluations/s",
                     "frac": cach / COLL_EVALS_PER_S, "kernel": "k_coll_blocks"}}
    print(f"[bench] linear basis: merge {merge_ms:.3f} ms ({ns} subsets), blocks {blocks_ms:.3f} ms "
          f"({nblk} blocks, {ach:.3e} evals/s = {100 * ach / peak:.1f}% of FP64 ceiling); collocation blocks "
          f"{coll_ms:.3f} ms ({cach:.3e} evals/s = {100 * cach / COLL_EVALS_PER_S:.1f}%, "
          f"Galerkin / collocation time {blocks_ms / coll_ms:.1f})", file=sys.stderr, flush=True)
    return res


def touching_pairs(mesh, rows):
    """Every pair (t, s), t in rows, s != t sharing a vertex with t, in both
    orders (unique)."""
    flat = mesh.tris.reshape(-1)
    order = np.argsort(flat, kind="stable")
    start = np.searchsorted(flat[order], np.arange(mesh.nv + 1))
    I, J = [], []
    for c in range(3):
        v = mesh.tris[rows, c]
        cnt = start[v + 1] - start[v]
        I.append(np.repeat(rows, cnt))
        J.append(np.concatenate([order[start[a]:start[a + 1]] for a in v]) // 3)
    I, J = np.concatenate(I), np.concatenate(J)
    pair = np.unique(np.stack([I, J], 1), axis=0)
    pair = pair[pair[:, 0] != pair[:, 1]]
    return np.concatenate([pair[:, 0], pair[:, 1]]), np.concatenate([pair[:, 1], pair[:, 0]])


def curved(gca, torch, mesh, nrows, steps=3, seed=13):
    """Curved (quadratic) triangles on the workload mesh (Section 6): edge
    points on the sphere, gca_curved_entries for the touching pairs of nrows
    random triangles (both orders; identical pairs added) and as many random
    pairs; single layer with the piecewise-constant basis (and the nodal
    moments, and the double layer), symmetric 6-point rule, q_s = 4; HIP events
    on the current stream around each call (no host work inside)."""
    import synth
    q = synth.quadratic(mesh, "sphere")
    rng = np.random.default_rng(seed)
    rows = rng.choice(mesh.nt, nrows, replace=False)
    Ti, Tj = touching_pairs(mesh, rows)
    Ti, Tj = np.concatenate([Ti, rows]), np.concatenate([Tj, rows])
    # regular pairs in blocks, as a block of the matrix presents them: 32 x 32
    # triangles of two patches (32 consecutive ids of the hierarchical mesh
    # numbering) whose centroids are at least 0.1 apart
    nb = Ti.size // 1024
    cen = mesh.verts[mesh.tris].mean(axis=1)
    pa = rng.integers(0, mesh.nt // 32, nb)
    pb = rng.integers(0, mesh.nt // 32, nb)
    far = np.linalg.norm(cen[32 * pa] - cen[32 * pb], axis=1) > 0.1
    pa, pb = pa[far], pb[far]
    loc = np.arange(32)
    Ri = (32 * pa[:, None, None] + loc[None, :, None] + 0 * loc[None, None, :]).reshape(-1)
    Rj = (32 * pb[:, None, None] + 0 * loc[None, :, None] + loc[None, None, :]).reshape(-1)
    shared = (mesh.tris[Ti][:, :, None] == mesh.tris[Tj][:, None, :]).sum(axis=(1, 2))
    qs, P = 4, 6
    regions = {1: 2, 2: 5, 3: 6}
    ss_evals = int(sum(regions[k] * np.count_nonzero(shared == k) for k in (1, 2, 3))) * qs ** 4
    nodes = torch.as_tensor(q.nodes, dtype=torch.float64).cuda()
    tri6 = torch.as_tensor(q.tris, dtype=torch.int32).cuda()
    dev = lambda a: torch.as_tensor(a.astype(np.int32)).cuda()
    sets = {"touching": (dev(Ti), dev(Tj)), "regular": (dev(Ri), dev(Rj))}
    res = {"workload": f"curved level-{int(round(math.log(mesh.nt / 20, 4)))} sphere ({q.nt} quadratic triangles, "
                       f"{q.nn} nodes, edge points projected onto the sphere); the touching pairs of {nrows} random "
                       f"triangles in both orders plus the identical pairs, and about as many regular pairs in 32 x 32 "
                       f"blocks of two patches of consecutive triangles at least 0.1 apart (seed {seed}); "
                       f"symmetric {P}-point rule, q_s = {qs}, FP64",
           "touching_classes": {"vertex": int(np.count_nonzero(shared == 1)),
                                "edge": int(np.count_nonzero(shared == 2)),
                                "identical": int(np.count_nonzero(shared == 3))}}
    for name, (I, J) in sets.items():
        out = {}
        for op, basis, key in ((0, 0, "single_constant"), (0, 1, "single_nodal"), (1, 0, "double_constant")):
            gca.curved_entries(nodes, tri6, I, J, op=op, basis=basis, q=3, sym=True, q_s=qs)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                gca.curved_entries(nodes, tri6, I, J, op=op, basis=basis, q=3, sym=True, q_s=qs)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            out[key] = {"ms": ms, "pairs_per_s": I.numel() / (ms * 1e-3)}
        out["pairs"] = int(I.numel())
        res[name] = out
    ms = res["regular"]["single_constant"]["ms"]
    ach = res["regular"]["pairs"] / (ms * 1e-3)
    res["regular"]["roofline"] = {"bound": "fp64 alu", "achieved": ach, "peak": curved_pairs_per_s(P),
                                  "unit": "pairs/s", "frac": ach / curved_pairs_per_s(P),
                                  "kernel": f"k_curved_regular<{P},0,0>"}
    ms = res["touching"]["single_constant"]["ms"]
    ach = ss_evals / (ms * 1e-3)
    res["touching"]["roofline"] = {"bound": "fp64 alu", "achieved": ach, "peak": CURVED_SS_EVALS_PER_S,
                                   "unit": "evaluations/s", "frac": ach / CURVED_SS_EVALS_PER_S,
                                   "evaluations": ss_evals, "kernel": "k_curved_touch<0,0>"}
    print(f"[bench] curved: {res['regular']['pairs']} regular pairs {ms_fmt(res['regular'])}; "
          f"{res['touching']['pairs']} touching pairs {ms_fmt(res['touching'])}; regular "
          f"{res['regular']['roofline']['frac']:.1%}, touching {res['touching']['roofline']['frac']:.1%} of the FP64 ceiling",
          file=sys.stderr, flush=True)
    return res


def ms_fmt(r):
    return ", ".join(f"{k} {v['ms']:.3f} ms" for k, v in r.items() if isinstance(v, dict) and "ms" in v)


# FP64 ceiling of one 4D Sauter-Schwab point of the double-layer touching
# pairs: the map and its weight (14 slots), the point difference (9), the
# kernel n . d |d|^-3 with the refined rsqrt and its quarter-rate v_rsq_f64
# (15), the weighted sum (1): 39 slots.
DL_SS_EVALS_PER_S = FP64_LANE_OPS_PER_S / 39.0


def double_layer(gca, torch, H, mesh, nrows, seed=11, steps=3):
    """Double-layer Galerkin entries (gca_dl_entries) on the workload mesh: the
    touching pairs (common vertex or edge) of nrows random triangles, both
    orders, and as many random pairs; HIP events on the current stream around
    each call (classification and integration on the device)."""
    rng = np.random.default_rng(seed)
    rows = rng.choice(mesh.nt, nrows, replace=False)
    Ti, Tj = touching_pairs(mesh, rows)
    Ri = rng.integers(0, mesh.nt, Ti.size)
    Rj = rng.integers(0, mesh.nt, Ti.size)
    shared = (mesh.tris[Ti][:, :, None] == mesh.tris[Tj][:, None, :]).sum(axis=(1, 2))
    qs = H.params.q_s
    evals = int(5 * np.count_nonzero(shared == 2) + 2 * np.count_nonzero(shared == 1)) * qs ** 4
    res = {"workload": f"touching pairs of {nrows} random triangles in both orders and as many random pairs "
                       f"(seed {seed}); FP64; HIP events around one gca_dl_entries call each"}
    for name, (a, b) in (("touching", (Ti, Tj)), ("random", (Ri, Rj))):
        I = torch.as_tensor(a.astype(np.int32)).cuda()
        J = torch.as_tensor(b.astype(np.int32)).cuda()
        out = torch.empty(I.numel(), dtype=torch.float64, device="cuda")
        call = lambda: gca._check(gca.lib().gca_dl_entries(H.h, ctypes_vp(I), ctypes_vp(J), I.numel(),
                                                           ctypes_vp(out), gca._stream_ptr(None)))
        call()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            call()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res[name] = {"pairs": int(a.size), "ms": ms, "entries_per_s": a.size / (ms * 1e-3)}
    ach = evals / (res["touching"]["ms"] * 1e-3)
    res["touching"]["roofline"] = {"bound": "fp64 alu", "achieved": ach, "peak": DL_SS_EVALS_PER_S,
                                   "unit": "evaluations/s", "frac": ach / DL_SS_EVALS_PER_S, "evaluations": evals,
                                   "kernel": "k_dl_pairs"}
    print(f"[bench] double layer: {res['touching']['pairs']} touching pairs in {res['touching']['ms']:.3f} ms "
          f"({res['touching']['roofline']['frac']:.1%} of the FP64 ceiling), {res['random']['pairs']} random pairs "
          f"in {res['random']['ms']:.3f} ms", file=sys.stderr, flush=True)
    return res


def ctypes_vp(t):
    import ctypes
    return ctypes.c_void_p(t.data_ptr())


def error_vectors(mesh, x_host):
    """The vectors of the error metric: the benchmark's x ~ N(0,1), the
    all-ones vector and the centroid x3 coordinate of every triangle (columns
    of an n x 3 array).  The smooth two load the far field, where the
    compression error lives."""
    c = mesh.verts[mesh.tris].mean(axis=1)
    return np.stack([x_host, np.ones(mesh.nt), c[:, 2]], axis=1)


def main():
    a = parse()
    if a.gpus != 1:
        sys.exit("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)")
    import torch
    import synth
    import paper_1810_08429_amd as gca

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    mesh, cfg = synth.workload(a.workload)
    n = mesh.nt
    if a.eps is not None:
        cfg["eps"] = a.eps
    if a.omega is not None:
        cfg["omega_scale"] = a.omega
    if a.green_m is not None:
        cfg["green_m"] = a.green_m
    print(f"[bench] workload {a.workload}: n={n} leaf={cfg['leaf']} eta={cfg['eta']} eps={cfg['eps']} "
          f"green_m={cfg['green_m']} omega={cfg.get('omega_scale', 0.25)}", file=sys.stderr, flush=True)
    params = gca.Params(eta=cfg["eta"], eps=cfg["eps"], green_m=cfg["green_m"],
                        omega_scale=cfg.get("omega_scale", 0.25))
    if a.q_c is not None:
        params.q_c = a.q_c
    elif "q_c" in cfg:
        params.q_c = cfg["q_c"]
    if a.q_nr is not None:
        params.q_nr = a.q_nr
    params.sym_rules = a.sym if a.sym is not None else cfg.get("sym_rules", 0)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tree = gca.Tree(mesh.verts, mesh.tris, cfg["leaf"])
    H = gca.H2(mesh.verts, mesh.tris, tree, params)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    st = H.stats()
    print(f"[bench] setup {setup_s:.2f} s (gca_build {st['build_ms'] / 1e3:.2f} s)", file=sys.stderr, flush=True)

    x_host = synth.rhs_normal(n, 1, seed=0)
    x = torch.tensor(x_host, device=dev)
    y = torch.empty_like(x)
    Xerr = torch.tensor(error_vectors(mesh, x_host), device=dev)

    def run(Hh, prec, steps, warmup):
        for _ in range(warmup):
            Hh.matvec_into(x, y, precision=prec)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            Hh.matvec_into(x, y, precision=prec)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        ph = Hh.phase_times(steps)
        return dt, ph, y.clone()

    if a.copy_probe:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] copy probe: 1 GiB read + 1 GiB written", file=sys.stderr, flush=True)
        del src, dst

    dt_mixed, ph_mixed, y_mixed = run(H, gca.MIXED, a.steps, a.warmup)
    print(f"[bench] mixed: {dt_mixed * 1e3:.3f} ms/product", file=sys.stderr, flush=True)
    fsteps = a.fp64_steps if a.fp64_steps is not None else max(3, a.steps // 2)
    dt_fp64, ph_fp64, y_fp64 = run(H, gca.FP64, fsteps, 1)
    print(f"[bench] fp64 : {dt_fp64 * 1e3:.3f} ms/product", file=sys.stderr, flush=True)
    # products of the three error vectors (outside the timed region)
    Y_err = {"mixed": H.matvec(Xerr, gca.MIXED).cpu().numpy(), "fp64": H.matvec(Xerr, gca.FP64).cpu().numpy()}

    # adjoint of the energy E = 1/2 x^T G~ x w.r.t. the vertex coordinates
    # (h2_bilinear_grad, frozen structure), mixed and FP64; the first call of
    # each precision sets up the adjoint's index maps and is not timed
    grad = {}
    if a.grad_steps > 0:
        gvec = {}
        for prec, name in ((gca.MIXED, "mixed"), (gca.FP64, "fp64")):
            dxyz = torch.zeros((mesh.nv, 3), dtype=torch.float64, device=dev)
            H.bilinear_grad(x, x, 0.5, dxyz, prec)
            gvec[name] = dxyz.clone()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(a.grad_steps):
                H.bilinear_grad(x, x, 0.5, dxyz, prec)
            torch.cuda.synchronize()
            grad[name] = {"ms_per_step": (time.perf_counter() - t) / a.grad_steps * 1e3, "steps": a.grad_steps}
            print(f"[bench] energy gradient {name}: {grad[name]['ms_per_step']:.3f} ms", file=sys.stderr,
                  flush=True)
            del dxyz
        d = gvec["mixed"] - gvec["fp64"]
        grad["mixed_vs_fp64"] = {
            "rel_diff_max": float(d.abs().max() / gvec["fp64"].abs().max()),
            "rel_diff_2": float(torch.linalg.norm(d) / torch.linalg.norm(gvec["fp64"])),
            "what": "dE/dX of E = 1/2 x^T G~ x, mixed against FP64, relative to the FP64 gradient"}
        print(f"[bench] energy gradient mixed vs fp64: {grad['mixed_vs_fp64']['rel_diff_max']:.2e} (max norm)",
              file=sys.stderr, flush=True)
        del gvec, d

    # the opt-in FP32 Sauter-Schwab loops (gca_params.ss_fp32 = 1): a second
    # handle on the same tree and parameters
    ss32 = None
    if a.ss32_steps > 0:
        p32 = gca.Params(**{k: getattr(params, k) for k in params.__dataclass_fields__})
        p32.ss_fp32 = 1
        H32 = gca.H2(mesh.verts, mesh.tris, tree, p32)
        dt32, ph32, _ = run(H32, gca.MIXED, a.ss32_steps, 2)
        pm32 = dict(zip(gca.PHASES, ph32.mean(axis=0).tolist()))
        Y_err["mixed_ss_fp32"] = H32.matvec(Xerr, gca.MIXED).cpu().numpy()
        H32.close()
        ss32 = {"value": n / dt32, "unit": "DoF/s", "ms_per_step": dt32 * 1e3, "steps": a.ss32_steps,
                "phases_ms": pm32,
                "phases_roofline_touching": phase_rooflines(st, params, rule_points(params.q_r, params.sym_rules),
                                                            rule_points(params.q_c, params.sym_rules), pm32,
                                                            ss_fp32=True)["touching"]}
        print(f"[bench] mixed with FP32 Sauter-Schwab loops: {dt32 * 1e3:.3f} ms/product", file=sys.stderr,
              flush=True)

    # the same product with every phase alone on the caller's stream
    # (gca_params.serial = 1): each kernel's duration without the others
    serial = None
    if a.serial_steps > 0:
        ps = gca.Params(**{k: getattr(params, k) for k in params.__dataclass_fields__})
        ps.serial = 1
        Hs = gca.H2(mesh.verts, mesh.tris, tree, ps)
        dts, phs, ys = run(Hs, gca.MIXED, a.serial_steps, 2)
        pms = dict(zip(gca.PHASES, phs.mean(axis=0).tolist()))
        serial = {"ms_per_step": dts * 1e3, "steps": a.serial_steps, "phases_ms": pms,
                  "bit_equal_to_overlapped": bool(torch.equal(ys, y_mixed))}
        Hs.close()
        print(f"[bench] mixed, phases serialised: {dts * 1e3:.3f} ms/product", file=sys.stderr, flush=True)

    # 16 right-hand sides in one call: every block entry evaluated once for
    # the 16 columns, transfer / coupling / nearfield products as matrix-core
    # tiles; against 16 single products of the same columns
    rhs16 = None
    if a.rhs16_steps > 0:
        # column-major n x 16 (leading dimension n), as h2_matvec takes them
        X16 = torch.tensor(synth.rhs_normal(n, 16, seed=1).T.copy(), device=dev).t()
        Y16 = torch.empty((16, n), dtype=torch.float64, device=dev).t()
        rhs16 = {"workload": "16 columns x ~ N(0,1) seed 1 in one h2_matvec call (nrhs = 16, ld = n)"}
        for prec, name, dt1 in ((gca.MIXED, "mixed", dt_mixed), (gca.FP64, "fp64", dt_fp64)):
            H.matvec_into(X16, Y16, precision=prec)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(a.rhs16_steps):
                H.matvec_into(X16, Y16, precision=prec)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t) / a.rhs16_steps
            ph = dict(zip(gca.PHASES, H.phase_times(a.rhs16_steps).mean(axis=0).tolist()))
            y0 = H.matvec(X16[:, 0].contiguous(), precision=prec)
            rhs16[name] = {"value": 16 * n / dt, "unit": "DoF/s", "ms_per_step": dt * 1e3, "steps": a.rhs16_steps,
                           "speedup_vs_16_single_products": 16 * dt1 / dt, "phases_ms": ph,
                           "rel_diff_column0_vs_single": float((Y16[:, 0] - y0).abs().max() / y0.abs().max())}
            print(f"[bench] 16 right-hand sides {name}: {dt * 1e3:.3f} ms ({16 * dt1 / dt:.1f}x 16 single products)",
                  file=sys.stderr, flush=True)
        del X16, Y16

    # stored-block mode: the block rows computed once (gca_store_blocks), then
    # products that read them; reported beside the recomputing product
    stored = {}
    if a.stored_steps > 0:
        torch.cuda.synchronize()
        t = time.perf_counter()
        H.store_blocks(fp64=True, mixed=True)
        torch.cuda.synchronize()
        t_store = time.perf_counter() - t
        st2 = H.stats()
        entries = st2["store_entries_far"] + st2["store_entries_near"]
        stored = {"store_s": t_store, "entries": entries,
                  "bytes": {"mixed": 4 * entries, "fp64": 8 * entries}}
        for prec, name, yref in ((gca.MIXED, "mixed", y_mixed), (gca.FP64, "fp64", y_fp64)):
            dt, ph, ys = run(H, prec, a.stored_steps, 2)
            pm = dict(zip(gca.PHASES, ph.mean(axis=0).tolist()))
            blk_ms = pm["coupling_blocks"] + pm["near_blocks"]
            stored[name] = {"value": n / dt, "unit": "DoF/s", "ms_per_step": dt * 1e3,
                            "block_rows_ms": blk_ms,
                            "block_rows_GBps": stored["bytes"][name] / (blk_ms * 1e-3) / 1e9,
                            "rel_diff_vs_recomputed": float(torch.linalg.norm(ys - yref) / torch.linalg.norm(yref)),
                            "phases_ms": pm}
            gbps = stored["bytes"][name] / (blk_ms * 1e-3) / 1e9
            stored[name]["roofline"] = {
                "bound": "hbm", "achieved": gbps, "peak": HBM_BYTES_PER_S / 1e9, "unit": "GB/s",
                "frac": gbps * 1e9 / HBM_BYTES_PER_S,
                "bytes": stored["bytes"][name], "kernel": "k_rows_apply",
                "timing": "the coupling and nearfield block-row launches (HIP events per phase), their times "
                          "added although they run on two streams at once, so a lower bound"}
            print(f"[bench] stored blocks {name}: {dt * 1e3:.3f} ms/product, block rows "
                  f"{stored[name]['block_rows_GBps']:.0f} GB/s", file=sys.stderr, flush=True)
        H.store_blocks(False, False)

    dl = double_layer(gca, torch, H, mesh, a.dl_rows) if a.dl_rows > 0 else None
    curv = curved(gca, torch, mesh, a.curved_rows) if a.curved_rows > 0 else None

    linear = None
    if a.lin_blocks > 0:
        linear = linear_basis(gca, torch, mesh, a.lin_blocks, max(a.stored_steps, 3), 2)
    nodal = lin_h2(gca, torch, a.nodal_level) if a.nodal_level > 0 else None
    solve = solve_leg(gca, torch, a.solve_steps) if a.solve_steps > 0 else None

    phases = gca.PHASES
    mean_mixed = dict(zip(phases, ph_mixed.mean(axis=0).tolist()))
    mean_fp64 = dict(zip(phases, ph_fp64.mean(axis=0).tolist()))

    # dominant kernel of the mixed product: coupling-block or nearfield-block quadrature
    P = rule_points(params.q_r, params.sym_rules)
    Pc = rule_points(params.q_c, params.sym_rules)
    work = {"coupling_blocks": st["coupling_entries"] * Pc * Pc * FLOPS_PER_EVAL,
            "near_blocks": st["near_regular_pairs"] * P * P * FLOPS_PER_EVAL}
    dom = max(work, key=lambda k: mean_mixed[k])
    dur = mean_mixed[dom] * 1e-3
    achieved = work[dom] / dur / 1e12
    kname = ("k_far_rows<float,%d>" % Pc) if dom == "coupling_blocks" else ("k_near_rows<float,%d>" % P)
    roofline = {"bound": "alu", "achieved": achieved, "peak": PUBLISHED_F32_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PUBLISHED_F32_TFLOPS, "traffic": measured_traffic(kname),
                "issue_ceiling": ISSUE_CEILING_F32_TFLOPS, "issue_ceiling_frac": achieved / ISSUE_CEILING_F32_TFLOPS,
                "kernel": kname, "phase": dom, "avg_ms": mean_mixed[dom], "flops_per_launch": work[dom],
                "timing": "HIP events around the kernel on its stream in the timed products, where the "
                          "transform chain and the touching lists run beside it on the handle's side streams"}
    if rhs16 is not None:
        # dominant kernel of the batched product: the nearfield block rows,
        # per unordered regular pair P^2 evaluations (10 flops each) and the
        # two 16-column products of the entry on the matrix cores (64 flops)
        for name in ("mixed", "fp64"):
            ms16 = rhs16[name]["phases_ms"]["near_blocks"]
            fl = st["near_regular_pairs"] * (P * P * FLOPS_PER_EVAL + 64)
            ach = fl / (ms16 * 1e-3) / 1e12
            pk = PUBLISHED_F32_TFLOPS if name == "mixed" else PUBLISHED_F64_TFLOPS
            rhs16[name]["roofline"] = {
                "bound": "alu", "achieved": ach, "peak": pk, "unit": "TFLOP/s", "frac": ach / pk, "flops": fl,
                "kernel": "k_near_rows_nb<%s,%d>" % ("float" if name == "mixed" else "double", P), "avg_ms": ms16,
                "timing": "HIP events around the kernel in the timed batched products (the transform chain and "
                          "the touching lists run beside it)"}
    if a.grad_steps > 0:
        # block derivatives of the adjoint: every ordered pair of the
        # nearfield and coupling blocks (both orientations), per evaluation
        # 18 flops (difference, |d|^2, w/r, its sum, w/r^3 and the 3-vector
        # accumulation; the rsqrt not counted)
        gev = 2 * (st["near_regular_pairs"] * P * P + st["coupling_entries"] * Pc * Pc)
        gfl = gev * GRAD_FLOPS_PER_EVAL
        ag = gfl / (grad["mixed"]["ms_per_step"] * 1e-3) / 1e12
        grad["roofline"] = {
            "bound": "alu", "achieved": ag, "peak": PUBLISHED_F32_TFLOPS, "unit": "TFLOP/s",
            "frac": ag / PUBLISHED_F32_TFLOPS, "evaluations": gev, "flops": gfl,
            "kernel": "k_grad_blocks<float,%d,true> and k_grad_blocks<float,%d,false>" % (P, Pc),
            "timing": "the whole mixed h2_bilinear_grad call (basis terms, pair lists and transforms "
                      "included), so a lower bound of the block kernels' own rate; their own times are "
                      "in the committed kernel trace of the gradient"}
    if serial is not None:
        a_ser = work[dom] / (serial["phases_ms"][dom] * 1e-3) / 1e12
        roofline["alone"] = {"avg_ms": serial["phases_ms"][dom], "achieved": a_ser,
                             "frac": a_ser / PUBLISHED_F32_TFLOPS,
                             "issue_ceiling_frac": a_ser / ISSUE_CEILING_F32_TFLOPS,
                             "timing": "the same kernel in the serial-phase products (gca_params.serial = 1)"}

    # CPU oracle on a bounded sample of rows (also the accuracy check): the
    # first rows of one seeded permutation, err_rows of them unless fewer fit
    # in about twice cpu_seconds, so runs of different configurations compare
    # on the same rows; the oracle computes the rows for the three error
    # vectors at once (the entries dominate its time)
    cpu = None
    rel = {}
    if a.cpu_seconds > 0:
        import oracle
        ent = oracle.Entries(mesh.verts, mesh.tris, params.q_r, params.q_nr, params.q_s)
        Xh = error_vectors(mesh, x_host)
        order = np.random.default_rng(12345).permutation(n)
        k0 = oracle.num_threads()
        rows = order[:k0]
        t = time.perf_counter()
        ref = ent.matvec_rows(rows, Xh)
        t1 = time.perf_counter() - t
        k = int(min(a.err_rows, max(k0, 2 * a.cpu_seconds / max(t1, 1e-6) * k0)))
        if k > k0:
            rows2 = order[k0:k]
            t = time.perf_counter()
            ref2 = ent.matvec_rows(rows2, Xh)
            t1 += time.perf_counter() - t
            rows = order[:k]
            ref = np.concatenate([ref, ref2])
        cpu = {"value": len(rows) / t1, "unit": "DoF/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"{len(rows)} rows of the dense FP64 product G X for 3 vectors at once (collapsed Gauss "
                         f"rules of the stated orders, Sauter-Schwab touching pairs), {t1:.1f} s; a full product "
                         f"is n rows, so DoF/s = rows/s"}
        names = ["x_normal", "ones", "x3"]
        for key, Y in Y_err.items():
            errs = {nm: float(np.linalg.norm(Y[rows, j] - ref[:, j]) / np.linalg.norm(ref[:, j]))
                    for j, nm in enumerate(names)}
            rel[key] = max(errs.values())
            rel[key + "_per_vector"] = errs
        rel["rows"] = int(len(rows))
        print(f"[bench] oracle rows {len(rows)} in {t1:.1f} s; rel err (max of x, 1, x3) mixed {rel['mixed']:.2e} "
              f"fp64 {rel['fp64']:.2e}; per vector mixed {rel['mixed_per_vector']}", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": n / dt_mixed,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt_mixed * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{a.workload}: unit icosphere, {n} flat triangles, piecewise-constant basis, "
                               f"leaf {cfg['leaf']}, eta {cfg['eta']}, Green order {cfg['green_m']}, "
                               f"omega margin {params.omega_scale} diam/eta, ACA eps {cfg['eps']}, "
                               f"Gauss orders regular {params.q_r} / coupling {params.q_c} / "
                               f"near {params.q_nr} / Sauter-Schwab {params.q_s}, "
                               f"disjoint-pair triangle rules "
                               f"{'symmetric' if params.sym_rules else 'collapsed Gauss'} ({P} points regular, {Pc} coupling), "
                               f"1 RHS x ~ N(0,1) seed 0",
                   "n": n, "nrhs": 1, "precision": "mixed: FP32 regular-pair quadrature + transfers, "
                                                   "FP64 Sauter-Schwab touching pairs"},
        "setup_s": setup_s,
        "setup_ms": {"tree": (setup_s * 1e3 - st["build_ms"]), **st["setup_ms"]},
        "fp64": {"value": n / dt_fp64, "unit": "DoF/s", "ms_per_step": dt_fp64 * 1e3, "steps": fsteps},
        "mixed_ss_fp32": ss32,
        "energy_gradient": grad,
        "stored_blocks": stored,
        "linear_basis": linear,
        "nodal_h2": nodal,
        "solve_level7": solve,
        "double_layer": dl,
        "curved": curv,
        "mixed_over_fp64": dt_fp64 / dt_mixed,
        "rel_err_sampled_rows": rel,
        "phases_ms": {"mixed": mean_mixed, "fp64": mean_fp64},
        "structure": {k: st[k] for k in ("n_clusters", "n_leaves", "depth", "n_far_sym", "n_near_sym",
                                         "n_ident", "n_edge", "n_vert", "n_nearreg", "coupling_entries",
                                         "near_regular_pairs", "rank_min", "rank_max", "rank_mean",
                                         "basis_bytes_fp64")},
        "roofline": roofline,
        "phases_roofline": phase_rooflines(st, params, P, Pc, mean_mixed),
        "serial_phases": serial,
        "multi_rhs16": rhs16,
        "phases_roofline_alone": (phase_rooflines(st, params, P, Pc, serial["phases_ms"])
                                  if serial is not None else None),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    H.close()


if __name__ == "__main__":
    main()
