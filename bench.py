"""Benchmark of the domain-decomposed ILU0 path on one MI355X.

One step = one pass of the whole path over the workload's matrix, already
resident in HBM: partition + reorder, drop + level sets + block ILU0/ILDU0,
BiCGSTAB to rel. residual 1e-8 with the FP64 preconditioner (once with every
apply timed by a HIP event pair, once untimed), FP32 factor copies, BiCGSTAB
to 1e-8 with FP32-stored factors and FP64 trisolve arithmetic (DD_MIXED;
timed and untimed), BiCGSTAB to 1e-8 with FP32 trisolves (DD_FP32, timed),
and, when trained parameters are present
(paper_2508_04917_amd/lic_params.npz), the learned interface correction:
faces + features + MLP inference, then BiCGSTAB to 1e-8 with the corrected
mixed-precision preconditioner.  Reported solve times are the untimed
solves' (no event records between the kernels).

Printed (one JSON line): the trisolve bandwidth of the FP64 apply -- its
algorithmic bytes divided by its average duration, timed by a HIP event
pair that the apply kernel's launch records at its start and end
(hipExtLaunchKernel, on the solve's stream) for every apply inside the
timed solve -- and its fraction of the 8 TB/s HBM peak, the BiCGSTAB times,
and the oracle's apply bandwidth on the same matrix (on the host's cores
and on one) as a CPU baseline.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
MALL_BYTES = 256 << 20  # MI355X last-level cache (Infinity Cache)
METRIC = "trisolve GB/s & %HBM peak; BiCGSTAB s to 1e-8: learned+FP32 vs plain FP64"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_sha(path):
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(workload, sub):
    """HBM bytes per apply from committed rocprofv3 counter runs, if they were
    taken on the current apply kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(workload)
    except (ValueError, OSError):
        return None
    if not rec or list(rec.get("subdomain", [])) != list(sub):
        return None
    src = os.path.join(ROOT, "paper_2508_04917_amd", "csrc", "apply.hip")
    if rec.get("apply_source_sha") != source_sha(src):
        return None
    return rec.get("bytes_per_apply")


def kernels_only(args, p, sub, ptr_d, col_d, val_d, dd, torch):
    """A plain device copy of known size (the reference for scaling hardware
    byte counters), then bursts of applies in each precision and of the
    SpMV, each burst timed with events on the stream the library launches
    on.  An apply whose bytes would stay in the last-level cache is also
    timed one apply at a time after a 1 GiB write."""
    import numpy as np
    copy_elems = 1 << 28  # 2 GiB of FP64 read + 2 GiB written
    src = torch.ones(copy_elems, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    out = {"copy_bytes_read": copy_elems * 8, "copy_bytes_written": copy_elems * 8}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for _ in range(2):
        dst.copy_(src)
    ev[0].record()
    for _ in range(3):
        dst.copy_(src)
    ev[1].record()
    torch.cuda.synchronize()
    out["copy_us"] = 1e3 * ev[0].elapsed_time(ev[1]) / 3
    out["copy_GBs"] = 2 * copy_elems * 8 / (out["copy_us"] * 1e-6) / 1e9
    del src, dst
    h = dd.dd_partition(p.nx, p.ny, p.nz, p.bs, ptr_d, col_d, val_d, sub=sub)
    dd.ilu0_factor(h, dd.DD_FP64)
    r = torch.randn(p.n * p.bs, dtype=torch.float64, device="cuda:0")
    z = torch.empty_like(r)
    for name, prec in (("fp64", dd.DD_FP64), ("mixed", dd.DD_MIXED), ("fp32", dd.DD_FP32)):
        dd.dd_set_precision(h, prec)
        dd.dd_trsv_apply(h, r, z)
        ev[0].record()
        for _ in range(args.applies):
            dd.dd_trsv_apply(h, r, z)
        ev[1].record()
        torch.cuda.synchronize()
        us = 1e3 * ev[0].elapsed_time(ev[1]) / args.applies
        nbytes = dd.dd_get_info(h)["apply_bytes"]
        out[name] = {"us_per_apply": round(us, 2), "bytes_per_apply": nbytes, "GB/s": round(nbytes / us / 1e3, 1)}
        log(f"{name}: {us:.1f} us per apply, {nbytes / us / 1e3:.1f} GB/s")
        if nbytes < MALL_BYTES:
            # the apply's working set fits the 256 MB last-level cache, so a
            # burst reads it from there (an effective rate, not HBM's): time
            # each apply again after writing 1 GiB, which evicts it
            flush = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0")
            fev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.applies)]
            for e in fev:
                flush.fill_(1.0)
                e[0].record()
                dd.dd_trsv_apply(h, r, z)
                e[1].record()
            torch.cuda.synchronize()
            fus = float(np.median([1e3 * e[0].elapsed_time(e[1]) for e in fev]))
            del flush
            out[name]["after_cache_flush"] = {"us_per_apply": round(fus, 2), "GB/s": round(nbytes / fus / 1e3, 1)}
            log(f"{name} after a cache flush: {fus:.1f} us per apply, {nbytes / fus / 1e3:.1f} GB/s")
    # the learned correction on FP32 factors (the metric's learned leg), with
    # the shipped parameters; bytes as the mixed apply's plus 64 per face
    # (C_f in FP32, the face's column and r_J)
    lic_path = os.path.join(ROOT, "paper_2508_04917_amd", "lic_params.npz")
    if p.bs == 3 and os.path.exists(lic_path):
        from paper_2508_04917_amd.lic import load_params
        dd.dd_set_precision(h, dd.DD_MIXED)
        dd.lic_setup(h)
        dd.lic_set_params(h, torch.as_tensor(load_params(lic_path)[0], device="cuda:0"))
        nf = dd.lic_get_faces(h)[0].numel()
        dd.dd_trsv_apply(h, r, z)
        ev[0].record()
        for _ in range(args.applies):
            dd.dd_trsv_apply(h, r, z)
        ev[1].record()
        torch.cuda.synchronize()
        us = 1e3 * ev[0].elapsed_time(ev[1]) / args.applies
        nbytes = dd.dd_get_info(h)["apply_bytes"] + 64 * nf
        out["learned_mixed"] = {"us_per_apply": round(us, 2), "bytes_per_apply": nbytes, "faces": nf,
                                "GB/s": round(nbytes / us / 1e3, 1)}
        log(f"learned_mixed: {us:.1f} us per apply, {nbytes / us / 1e3:.1f} GB/s")
        dd.lic_set_params(h, None)
        dd.dd_set_precision(h, dd.DD_FP64)
    # SpMV bursts on the layout the handle uses; bytes as the BSR count
    # (FP64 blocks, int32 columns and row pointers, x once, y)
    info = dd.dd_get_info(h)
    dd.dd_spmv(h, r, z)
    ev[0].record()
    for _ in range(args.applies):
        dd.dd_spmv(h, r, z)
    ev[1].record()
    torch.cuda.synchronize()
    us = 1e3 * ev[0].elapsed_time(ev[1]) / args.applies
    bb = info["bs"] * info["bs"]
    nbytes = info["nnzb"] * (bb * 8 + 4) + (info["n"] + 1) * 4 + 2 * info["n"] * info["bs"] * 8
    layout = {0: "CSR", 1: "sliced ELL", 2: "sliced ELL, one width per slice",
              3: "sliced ELL per part, x in LDS"}[info["spmv_layout"]]
    out["spmv"] = {"us_per_call": round(us, 2), "layout": layout, "bytes_per_call": nbytes,
                   "GB/s": round(nbytes / us / 1e3, 1)}
    log(f"spmv: {us:.1f} us per call, {nbytes / us / 1e3:.1f} GB/s")
    h.close()
    print(json.dumps(out), flush=True)


ABLATIONS = {
    1: "plain level loop (reference for 4-8)",
    4: "split: lower + diagonal scaling, then upper, two kernels",
    5: "vector in global memory instead of LDS",
    6: "vertex-centric: one thread per block row",
    7: "ILU0 form: unscaled U, row sums scaled by inv(U_II)",
    8: "synchronisation-free sweeps, per-row flags in LDS (Algorithm 4)",
    3: "production: slot layout, hand-scheduled prefetch",
}


def ablation(args, p, sub, ptr_d, col_d, val_d, dd, torch):
    """FP64 apply kernel variants on the same factors: bursts of applies per
    variant, timed with events, outputs compared with the production
    kernel's.  Bytes are the method's algorithmic bytes per apply for all
    variants (the same factors and vectors are needed by each)."""
    h = dd.dd_partition(p.nx, p.ny, p.nz, p.bs, ptr_d, col_d, val_d, sub=sub)
    dd.ilu0_factor(h, dd.DD_FP64)
    nbytes = dd.dd_get_info(h)["apply_bytes"]
    g = torch.Generator(device="cuda:0")
    g.manual_seed(11)
    r = torch.randn(p.n * p.bs, dtype=torch.float64, device="cuda:0", generator=g)
    z = torch.empty_like(r)
    ref = torch.empty_like(r)
    dd.dd_set_apply_variant(h, 3)
    dd.dd_trsv_apply(h, r, ref)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    inf = dd.dd_get_info(h)
    out = {"workload": args.workload, "subdomain": [inf["sx"], inf["sy"], inf["sz"]], "n_subdomains": inf["nsub"],
           "bytes_per_apply": nbytes, "applies": args.applies, "variants": {}}
    for v, what in ABLATIONS.items():
        log(f"variant {v}: {what}")
        dd.dd_set_apply_variant(h, v)
        dd.dd_trsv_apply(h, r, z)
        ev[0].record()
        for _ in range(args.applies):
            dd.dd_trsv_apply(h, r, z)
        ev[1].record()
        torch.cuda.synchronize()
        us = 1e3 * ev[0].elapsed_time(ev[1]) / args.applies
        diff = float(torch.linalg.vector_norm(z - ref) / torch.linalg.vector_norm(ref))
        out["variants"][str(v)] = {"what": what, "us_per_apply": round(us, 2),
                                   "GB/s": round(nbytes / us / 1e3, 1), "rel_diff_vs_variant3": diff}
        log(f"  {us:.1f} us per apply, {nbytes / us / 1e3:.1f} GB/s, rel diff {diff:.1e}")
    dd.dd_set_apply_variant(h, 0)
    h.close()
    print(json.dumps(out), flush=True)


def rocsparse_scalar(p, ptr, col, val, r, z_ref, burst, rel, us_dd):
    """rocSPARSE's scalar ILU0 (csrilu0, csrsv) on the CSR expansion of a
    BSR matrix: the same preconditioner on a pattern of dense blocks."""
    import torch
    from paper_2508_04917_amd.rocsparse_ref import RocsparseILU0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rs = RocsparseILU0(p.n, p.bs, ptr, col, val, scalar=True)
    setup = time.perf_counter() - t0
    zs = torch.empty_like(r)
    us_rs = burst(lambda: rs.apply(r, zs))
    rs.close()
    res = {"us": round(us_rs, 2), "setup_s": round(setup, 3), "rel_diff": rel(zs, z_ref),
           "dd_apply_speedup": round(us_rs / us_dd, 2)}
    log(f"  rocSPARSE scalar ILU0 (CSR expansion): {us_rs:.1f} us per apply ({us_rs / us_dd:.1f}x the DD apply), "
        f"setup {setup:.2f} s, rel diff {res['rel_diff']:.1e}")
    return res


def rocsparse_permuted(p, ptr, col, val, n2o, r, z_ref, burst, rel, us_dd):
    """rocSPARSE's ILU0 apply on P A P^T for the renumbering n2o (new ->
    old block rows), timed like the others; its output, renumbered back, is
    compared with z_ref (the apply of the same factors in the old order)."""
    import torch
    from paper_2508_04917_amd.rocsparse_ref import RocsparseILU0, permuted_matrix
    pp, pc, pv = permuted_matrix(ptr, col, val, n2o, p.bs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rs = RocsparseILU0(p.n, p.bs, pp, pc, pv)
    setup = time.perf_counter() - t0
    rp = r.view(-1, p.bs)[n2o].reshape(-1).contiguous()
    zp = torch.empty_like(r)
    us_rs = burst(lambda: rs.apply(rp, zp))
    zb = torch.empty_like(r)
    zb.view(-1, p.bs)[n2o] = zp.view(-1, p.bs)
    rs.close()
    res = {"us": round(us_rs, 2), "setup_s": round(setup, 3), "rel_diff": rel(zb, z_ref),
           "dd_apply_speedup": round(us_rs / us_dd, 2)}
    log(f"  rocSPARSE ILU0, rows in level order: {us_rs:.1f} us per apply ({us_rs / us_dd:.1f}x the DD apply), "
        f"rel diff {res['rel_diff']:.1e}")
    return res


def rocsparse_cmp(args, p, sub, ptr_d, col_d, val_d, dd, torch):
    """The paper's headline comparison (Section 5.2, Table 4) restated on this
    GPU: rocSPARSE's block ILU0 apply (two block triangular solves) as a black
    box, on the decomposed matrix (the same preconditioner as the DD apply)
    and on the full matrix (global ILU0, against this library's
    level-scheduled global ILU0), outputs compared, bursts of applies timed
    with events."""
    from paper_2508_04917_amd.rocsparse_ref import RocsparseILU0, dropped_matrix, level_order
    h = dd.dd_partition(p.nx, p.ny, p.nz, p.bs, ptr_d, col_d, val_d, sub=sub)
    dd.ilu0_factor(h, dd.DD_FP64)
    inf = dd.dd_get_info(h)
    S = inf["sx"] * inf["sy"] * inf["sz"]
    nbytes = inf["apply_bytes"]
    g = torch.Generator(device="cuda:0")
    g.manual_seed(13)
    r = torch.randn(p.n * p.bs, dtype=torch.float64, device="cuda:0", generator=g)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def burst(fn):
        fn()
        ev[0].record()
        for _ in range(args.applies):
            fn()
        ev[1].record()
        torch.cuda.synchronize()
        return 1e3 * ev[0].elapsed_time(ev[1]) / args.applies

    def rel(a, b):
        return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))

    out = {"workload": args.workload, "subdomain": [inf["sx"], inf["sy"], inf["sz"]],
           "n_subdomains": inf["nsub"], "applies": args.applies}
    z = torch.empty_like(r)
    us = burst(lambda: dd.dd_trsv_apply(h, r, z))
    out["dd_apply"] = {"us": round(us, 2), "GB/s": round(nbytes / us / 1e3, 1)}
    log(f"DD-ILU0 apply: {us:.1f} us")

    ptr, col, val = dd.dd_get_reordered(h)
    ptr_t, col_t, val_t = dropped_matrix(ptr, col, val, S, p.bs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rs = RocsparseILU0(p.n, p.bs, ptr_t, col_t, val_t)
    setup = time.perf_counter() - t0
    z_rs = torch.empty_like(r)
    us_rs = burst(lambda: rs.apply(r, z_rs))
    out["rocsparse_decomposed"] = {"us": round(us_rs, 2), "setup_s": round(setup, 3),
                                   "rel_diff_vs_dd_apply": rel(z_rs, z),
                                   "dd_apply_speedup": round(us_rs / us, 2)}
    log(f"rocSPARSE ILU0 on the decomposed matrix: {us_rs:.1f} us per apply ({us_rs / us:.1f}x the DD apply), "
        f"setup {setup:.2f} s, rel diff {rel(z_rs, z):.1e}")
    rs.close()
    # the same matrix with its block rows sorted by level (every coupled pair
    # keeps its order, so the factors are the same): the ordering under which
    # a row-by-row triangular solve meets ready rows one after another
    n2o = level_order(ptr_t, col_t)
    out["rocsparse_decomposed_level_order"] = rocsparse_permuted(p, ptr_t, col_t, val_t, n2o, r, z, burst, rel, us)
    out["rocsparse_decomposed_scalar"] = rocsparse_scalar(p, ptr_t, col_t, val_t, r, z, burst, rel, us)
    del ptr_t, col_t, val_t

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dd.dd_global_factor(h)
    torch.cuda.synchronize()
    gsetup = time.perf_counter() - t0
    zg = torch.empty_like(r)
    us_g = burst(lambda: dd.dd_global_apply(h, r, zg))
    t0 = time.perf_counter()
    rsg = RocsparseILU0(p.n, p.bs, ptr, col, val)
    setup = time.perf_counter() - t0
    z_rsg = torch.empty_like(r)
    us_rsg = burst(lambda: rsg.apply(r, z_rsg))
    out["global_ilu0"] = {"this_library_us": round(us_g, 2), "this_library_setup_s": round(gsetup, 3),
                          "rocsparse_us": round(us_rsg, 2), "rocsparse_setup_s": round(setup, 3),
                          "rel_diff": rel(z_rsg, zg), "dd_apply_speedup_vs_rocsparse": round(us_rsg / us, 2)}
    log(f"global ILU0: this library {us_g:.1f} us, rocSPARSE {us_rsg:.1f} us per apply, rel diff {rel(z_rsg, zg):.1e}")
    rsg.close()
    # rocSPARSE on the matrix as given (natural grid order, no reordering):
    # the plain baseline a user of the vendor library would run
    t0 = time.perf_counter()
    rsn = RocsparseILU0(p.n, p.bs, ptr_d, col_d, val_d)
    setup = time.perf_counter() - t0
    z_rsn = torch.empty_like(r)
    us_rsn = burst(lambda: rsn.apply(r, z_rsn))
    out["rocsparse_natural_order"] = {"us": round(us_rsn, 2), "setup_s": round(setup, 3),
                                      "dd_apply_speedup": round(us_rsn / us, 2)}
    log(f"rocSPARSE ILU0 on the matrix in natural order: {us_rsn:.1f} us per apply ({us_rsn / us:.1f}x the DD apply)")
    rsn.close()
    # the natural order's global ILU0 with the rows sorted by level (the
    # grid's diagonal planes), checked against rocSPARSE's own apply in the
    # natural order (the same factors)
    n2o = level_order(ptr_d, col_d)
    out["rocsparse_natural_level_order"] = rocsparse_permuted(p, ptr_d, col_d, val_d, n2o, r, z_rsn, burst, rel, us)
    h.close()
    print(json.dumps(out), flush=True)


def graph_mode(args, p, ptr_d, col_d, val_d, dd, torch):
    """A matrix without geometry: graph partition (recursive BFS bisection,
    automatic part size), factor, bursts of FP64 applies, and BiCGSTAB to
    rtol, each timed."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = dd.dd_partition_graph(p.n, p.bs, ptr_d, col_d, val_d, part_rows=args.part_rows)
    torch.cuda.synchronize()
    t_part = time.perf_counter() - t0
    dd.ilu0_factor(h, dd.DD_FP64)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    inf = dd.dd_get_info(h)
    nbytes = inf["apply_bytes"]
    r = torch.randn(p.n * p.bs, dtype=torch.float64, device="cuda:0")
    z = torch.empty_like(r)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    dd.dd_trsv_apply(h, r, z)
    ev[0].record()
    for _ in range(args.applies):
        dd.dd_trsv_apply(h, r, z)
    ev[1].record()
    torch.cuda.synchronize()
    us = 1e3 * ev[0].elapsed_time(ev[1]) / args.applies
    y = torch.empty_like(r)
    dd.dd_spmv(h, r, y)
    ev[0].record()
    for _ in range(args.applies):
        dd.dd_spmv(h, r, y)
    ev[1].record()
    torch.cuda.synchronize()
    spmv_us = 1e3 * ev[0].elapsed_time(ev[1]) / args.applies
    b = torch.as_tensor(p.b, device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, info = dd.bicgstab_solve(h, b, rtol=args.rtol, maxit=args.maxit)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    out = {"workload": args.workload, "block_rows": p.n, "blocks": p.nnzb, "bs": p.bs,
           "part_rows": inf["S"], "n_subdomains": inf["nsub"], "dropped_blocks": p.nnzb - inf["nnzb_dropped"],
           "max_levels": list(inf["max_levels"]), "partition_s": round(t_part, 3),
           "setup_s": round(t_setup, 3), "apply_us": round(us, 2), "apply_bytes": nbytes,
           "apply_GB/s": round(nbytes / us / 1e3, 1), "spmv_us": round(spmv_us, 2),
           "spmv_layout": inf["spmv_layout"], "max_row_blocks": inf["max_row_blocks"],
           "bicgstab": {"iters": info["iters"], "status": info["status"],
                        "solve_s": round(info["solve_seconds"], 4), "call_wall_s": round(t_solve, 4),
                        "rel_res_true": info["rel_res_true"]}}
    log(f"graph partition {t_part:.3f} s, setup {t_setup:.3f} s, apply {us:.1f} us "
        f"({nbytes / us / 1e3:.1f} GB/s), BiCGSTAB {info['iters']} it {info['solve_seconds']:.3f} s "
        f"({t_solve:.3f} s for the first call, with its workspace allocation)")
    h.close()
    print(json.dumps(out), flush=True)


def precision_mode(args, p, sub, ptr_d, col_d, val_d, lic_params, dd, torch):
    """What the reduced-precision applies do to the preconditioner on this
    workload: each apply's error against the FP64 apply (in norm and per
    block row), its departure from linearity (M(a+b) - Ma - Mb and
    M(2a) - 2Ma, relative to the result; zero up to rounding for a linear
    operator), the variation between two applies of the same vector
    (repeatability), and BiCGSTAB with each precision, with and without
    the learned correction."""
    h = dd.dd_partition(p.nx, p.ny, p.nz, p.bs, ptr_d, col_d, val_d, sub=sub)
    dd.ilu0_factor(h, dd.DD_FP64)
    m = p.n * p.bs
    g = torch.Generator(device="cuda:0")
    g.manual_seed(11)
    a = torch.randn(m, dtype=torch.float64, device="cuda:0", generator=g)
    b = torch.randn(m, dtype=torch.float64, device="cuda:0", generator=g)
    b_d = torch.as_tensor(p.b, device="cuda:0")
    out = {"workload": args.workload, "subdomain": list(sub)}

    def rel(x, y):
        return float(torch.linalg.norm(x - y) / torch.linalg.norm(y))

    def rowmax(x, y):  # largest per-block-row error relative to the row's norm in y
        d = (x - y).view(-1, p.bs).norm(dim=1)
        n = y.view(-1, p.bs).norm(dim=1)
        return float((d / n.clamp_min(1e-300)).max())

    if lic_params is not None:
        dd.lic_setup(h)
    dd.dd_set_precision(h, dd.DD_FP64)
    z64 = dd.dd_trsv_apply(h, a)
    for name, prec in (("fp64", dd.DD_FP64), ("mixed", dd.DD_MIXED), ("fp32", dd.DD_FP32)):
        dd.dd_set_precision(h, prec)
        za = dd.dd_trsv_apply(h, a)
        za2 = dd.dd_trsv_apply(h, a)
        zb = dd.dd_trsv_apply(h, b)
        zab = dd.dd_trsv_apply(h, a + b)
        z2a = dd.dd_trsv_apply(h, 2.0 * a)
        zs = dd.dd_trsv_apply(h, 1e-3 * a)
        rec = {"apply_rel_err_vs_fp64": rel(za, z64), "apply_max_row_rel_err_vs_fp64": rowmax(za, z64),
               "additivity_defect": rel(zab, za + zb), "scaling_defect_x2": rel(z2a, 2.0 * za),
               "scaling_defect_x1e-3": rel(zs, 1e-3 * za), "repeat_identical": bool(torch.equal(za, za2))}
        for label, lic in (("plain", None), ("learned", lic_params)):
            if lic is None and label == "learned":
                continue
            dd.lic_set_params(h, lic)
            x, info = dd.bicgstab_solve(h, b_d, rtol=args.rtol, maxit=args.maxit)
            rec[f"bicgstab_{label}"] = {"iters": info["iters"], "status": info["status"],
                                        "solve_s": round(info["solve_seconds"], 4), "restarts": info["restarts"],
                                        "rel_res_true": info["rel_res_true"], "fallback": info["fallback"]}
            dd.lic_set_params(h, None)
        out[name] = rec
        log(f"{name}: {rec}")
    h.close()
    print(json.dumps(out), flush=True)


def dd_vs_global(args, p, subs, ptr_d, col_d, val_d, dd, torch):
    """What the decomposition costs and buys on one matrix (the comparison of
    Section 5.3, Tables 6 and 7, there against a rocSPARSE-based solver):
    BiCGSTAB to rtol with the DD-ILU0 preconditioner and with the global
    (undecomposed) ILU0 of the same reordered matrix, this library's
    level-scheduled kernels (one launch per level, vector in global memory),
    for each subdomain shape in subs: setup, apply and solve times and
    iteration counts."""
    b = torch.as_tensor(p.b, device="cuda:0")
    r = torch.randn(p.n * p.bs, dtype=torch.float64, device="cuda:0")
    z = torch.empty_like(r)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def burst(fn, k):
        fn()
        ev[0].record()
        for _ in range(k):
            fn()
        ev[1].record()
        torch.cuda.synchronize()
        return 1e3 * ev[0].elapsed_time(ev[1]) / k

    rows = []
    for sub in subs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = dd.dd_partition(p.nx, p.ny, p.nz, p.bs, ptr_d, col_d, val_d, sub=sub)
        dd.ilu0_factor(h, dd.DD_FP64)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        inf = dd.dd_get_info(h)
        us = burst(lambda: dd.dd_trsv_apply(h, r, z), args.applies)
        x, i_dd = dd.bicgstab_solve(h, b, rtol=args.rtol, maxit=args.maxit)
        log(f"{p.name} {inf['sx']}x{inf['sy']}x{inf['sz']}: DD-ILU0 setup {setup:.3f} s, apply {us:.1f} us, "
            f"BiCGSTAB {i_dd['iters']} it {i_dd['solve_seconds']:.3f} s")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dd.dd_global_factor(h)
        torch.cuda.synchronize()
        gsetup = time.perf_counter() - t0
        gus = burst(lambda: dd.dd_global_apply(h, r, z), max(2, args.applies // 5))
        dd.dd_set_preconditioner(h, 1)
        x, i_g = dd.bicgstab_solve(h, b, rtol=args.rtol, maxit=args.maxit)
        dd.dd_set_preconditioner(h, 0)
        log(f"{p.name}: global ILU0 setup {gsetup:.3f} s, apply {gus:.1f} us, "
            f"BiCGSTAB {i_g['iters']} it {i_g['solve_seconds']:.3f} s")
        rows.append({"subdomain": [inf["sx"], inf["sy"], inf["sz"]], "n_subdomains": inf["nsub"],
                     "blocks": inf["nnzb"], "blocks_after_drop": inf["nnzb_dropped"],
                     "dd_ilu0": {"setup_s": round(setup, 3), "apply_us": round(us, 2), "iters": i_dd["iters"],
                                 "status": i_dd["status"], "solve_s": round(i_dd["solve_seconds"], 4),
                                 "rel_res_true": i_dd["rel_res_true"]},
                     "global_ilu0": {"setup_s": round(gsetup, 3), "apply_us": round(gus, 2), "iters": i_g["iters"],
                                     "status": i_g["status"], "solve_s": round(i_g["solve_seconds"], 4),
                                     "rel_res_true": i_g["rel_res_true"]},
                     "iteration_ratio": round(i_dd["iters"] / max(1, i_g["iters"]), 3),
                     "solve_speedup": round(i_g["solve_seconds"] / max(1e-9, i_dd["solve_seconds"]), 2)})
        h.close()
    print(json.dumps({"workload": args.workload, "block_rows": p.n, "rtol": args.rtol, "rows": rows}), flush=True)


def host_cpu():
    """(model name, threads available to this process)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_baseline(args, p, sub, bytes64, np, gpu_iters=None):
    """The oracle timed on this host's CPU cores, on the same matrix: the
    DD-ILU0 apply single-threaded (the oracle's own whole-matrix call) and
    subdomain-parallel on every available core (one oracle call per
    subdomain's rows of the dropped matrix, which share no coupling; the
    calls release the GIL), bytes counted as for the GPU apply; plus the
    oracle's BiCGSTAB (setup and solve, single-threaded) on the 16^3 scalar
    Laplacian and the 64^3 random-block operator, and a few iterations of
    it on the same matrix (seconds per iteration, and the solve time that
    rate gives at the GPU solve's iteration count)."""
    import concurrent.futures as cf

    import oracle as O
    from problems import make_workload
    model, threads = host_cpu()
    log(f"cpu baseline: oracle setup on {p.nx}x{p.ny}x{p.nz} ({threads} threads of {model})")
    t = time.perf_counter()
    st = O.setup(p, tuple(sub))
    setup_s = time.perf_counter() - t
    r = np.random.default_rng(0).standard_normal(p.n * p.bs)
    st.apply(r)
    t = time.perf_counter()
    for _ in range(args.cpu_applies):
        st.apply(r)
    dt1 = (time.perf_counter() - t) / args.cpu_applies
    # per-subdomain slices of the dropped matrix and its factors (local columns)
    S, bs, bb = st.S, st.bs, st.bs * st.bs
    f = np.asarray(st.f).reshape(-1, bb)
    parts = []
    for k in range(st.nsub):
        a, b = int(st.tptr[k * S]), int(st.tptr[(k + 1) * S])
        ptr = (st.tptr[k * S:(k + 1) * S + 1] - a).astype(np.int32)
        col = (st.tcol[a:b] - k * S).astype(np.int32)
        parts.append((ptr, col, np.ascontiguousarray(f[a:b]), k * S * bs))
    z = np.empty_like(r)

    def one(part):
        ptr, col, fk, off = part
        z[off:off + S * bs] = O.apply(S, bs, ptr, col, fk, r[off:off + S * bs])

    with cf.ThreadPoolExecutor(max_workers=threads) as pool:
        list(pool.map(one, parts))
        zref = st.apply(r)
        assert np.array_equal(z, zref), "subdomain-parallel oracle apply differs from the whole-matrix call"
        t = time.perf_counter()
        for _ in range(args.cpu_applies):
            list(pool.map(one, parts))
        dtn = (time.perf_counter() - t) / args.cpu_applies
    out = {"value": round(bytes64 / dtn / 1e9, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
           "sample": f"{args.cpu_applies} oracle DD-ILU0 applies (FP64) on the full {p.nx}x{p.ny}x{p.nz} matrix "
                     f"on {threads} threads (one oracle call per subdomain), {dtn * 1e3:.1f} ms each; "
                     f"single-threaded {dt1 * 1e3:.1f} ms each; bytes counted as for the GPU apply",
           "cpu_model": model, "single_thread_GBs": round(bytes64 / dt1 / 1e9, 3),
           "apply_ms": {"threads": round(dtn * 1e3, 2), "single": round(dt1 * 1e3, 2)},
           "setup_s": round(setup_s, 3), "solves": {}}
    log(f"cpu baseline apply: {dt1 * 1e3:.1f} ms single-threaded, {dtn * 1e3:.1f} ms on {threads} threads")
    if args.cpu_iters > 0:
        # the oracle's BiCGSTAB (single-threaded) for a bounded number of
        # iterations on the bench matrix: its full solve would take minutes
        t = time.perf_counter()
        res = st.bicgstab(p.b, rtol=args.rtol, maxit=args.cpu_iters)
        t_it = (time.perf_counter() - t) / max(res.iters, 1)
        out["bicgstab"] = {"iterations_run": res.iters, "s_per_iteration": round(t_it, 3), "threads": 1}
        if gpu_iters:
            out["bicgstab"]["solve_s_at_gpu_iterations"] = round(t_it * gpu_iters, 1)
            out["bicgstab"]["gpu_iterations"] = gpu_iters
        log(f"cpu baseline BiCGSTAB on {p.nx}x{p.ny}x{p.nz}: {res.iters} iterations, {t_it:.2f} s each")
    if args.cpu_solves:
        for wname in ("laplacian16_scalar", "random64_bsr3"):
            q = make_workload(wname)
            qsub = WORKLOAD_SUB.get(wname)
            t = time.perf_counter()
            qs = O.setup(q, qsub)
            t_setup = time.perf_counter() - t
            t = time.perf_counter()
            res = qs.bicgstab(q.b, rtol=args.rtol)
            t_solve = time.perf_counter() - t
            out["solves"][wname] = {"iters": res.iters, "status": res.status, "setup_s": round(t_setup, 3),
                                    "solve_s": round(t_solve, 3), "subdomain": list(qsub), "threads": 1}
            log(f"cpu baseline {wname}: oracle setup {t_setup:.2f} s, BiCGSTAB {res.iters} it {t_solve:.2f} s")
    return out


# subdomain extents of the oracle solves in the CPU baseline: those the GPU
# library chooses for the workload on an MI355X (160 KB of LDS, 256 CUs)
WORKLOAD_SUB = {"laplacian16_scalar": (8, 8, 8), "random64_bsr3": (8, 8, 16)}


def compare_workload(args, wname, override, lic_params, dd, torch, np):
    """One more workload, outside the timed steps: BiCGSTAB to rtol with plain
    FP64 DD-ILU0, with FP32-stored factors (DD_MIXED), and with the learned
    correction + FP32-stored factors; iterations, solve seconds, the
    library's true residual and the residual of each solution recomputed by
    the oracle's FP64 SpMV on the matrix as generated."""
    import oracle as O
    from problems import make_workload
    log(f"extra workload {wname}: generating")
    q = make_workload(wname, **override)
    dev = "cuda:0"
    ptr_d = torch.as_tensor(q.brow_ptr, device=dev)
    col_d = torch.as_tensor(q.bcol, device=dev)
    val_d = torch.as_tensor(q.val.reshape(-1), device=dev)
    b_d = torch.as_tensor(q.b, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = dd.dd_partition(q.nx, q.ny, q.nz, q.bs, ptr_d, col_d, val_d)
    dd.ilu0_factor(h, dd.DD_FP64)
    torch.cuda.synchronize()
    inf = dd.dd_get_info(h)
    rec = {"grid": [q.nx, q.ny, q.nz], "seed": q.seed, "subdomain": [inf["sx"], inf["sy"], inf["sz"]],
           "n_subdomains": inf["nsub"], "setup_s": round(time.perf_counter() - t0, 4)}
    bn = float(np.linalg.norm(q.b))

    def solve(label):
        x, info = dd.bicgstab_solve(h, b_d, rtol=args.rtol, maxit=args.maxit)
        xs = x.cpu().numpy()
        res_o = float(np.linalg.norm(O.spmv(q.n, q.bs, q.brow_ptr, q.bcol, q.val, xs) - q.b) / bn)
        rec[label] = {"iters": info["iters"], "status": info["status"], "solve_s": round(info["solve_seconds"], 4),
                      "rel_res_true": info["rel_res_true"], "oracle_rel_res": res_o,
                      "restarts": info["restarts"], "fallback": info["fallback"]}
        log(f"  {wname} {label}: {info['iters']} it, {info['solve_seconds']:.3f} s, "
            f"oracle residual {res_o:.2e}")
        return x

    solve("plain_fp64")
    dd.dd_set_precision(h, dd.DD_MIXED)
    solve("mixed_fp32_factors")
    if lic_params is not None and q.bs == 3:
        t = time.perf_counter()
        dd.lic_setup(h)
        dd.lic_set_params(h, lic_params)
        torch.cuda.synchronize()
        rec["lic_setup_s"] = round(time.perf_counter() - t, 4)
        solve("learned_mixed")
        dd.lic_set_params(h, None)
    h.close()
    p64, pl = rec["plain_fp64"], rec.get("learned_mixed")
    if pl:
        rec["learned_mixed_speedup_vs_plain_fp64"] = round(p64["solve_s"] / pl["solve_s"], 3)
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lognormal160_bsr3")
    ap.add_argument("--sub", default="auto", help="sx,sy,sz or auto")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=5000)
    ap.add_argument("--cpu-applies", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=2,
                    help="iterations of the oracle's BiCGSTAB timed on the bench matrix (0: none)")
    ap.add_argument("--cpu-solves", type=int, default=1,
                    help="1: the CPU baseline also times the oracle's BiCGSTAB on the 16^3 scalar "
                         "and 64^3 random-block workloads")
    ap.add_argument("--extra", type=int, default=1,
                    help="1: after the timed steps, compare plain FP64, FP32-factor and learned solves on "
                         "the anisotropic 160^3 and the 128^3 evaluation workloads")
    ap.add_argument("--mode", default="full",
                    choices=["full", "kernels", "ablation", "rocsparse", "graph", "precision", "global"],
                    help="kernels: only a copy kernel of known size and bursts of applies and SpMVs "
                         "(the short program the rocprofv3 counter runs profile); "
                         "ablation: the FP64 apply kernel variants, timed on the same factors; "
                         "rocsparse: rocSPARSE's block ILU0 apply on the decomposed and the full matrix; "
                         "graph: graph partition, apply and solve of a workload without geometry; "
                         "precision: error, nonlinearity and solves of the FP32-factor applies; "
                         "global: BiCGSTAB with DD-ILU0 against the global ILU0 of the same matrix "
                         "(the workload's subdomains, then the automatic ones)")
    ap.add_argument("--applies", type=int, default=10)
    ap.add_argument("--part-rows", type=int, default=0,
                    help="graph mode: rows per part (0: the library's automatic choice)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the apply and the solver run on one GPU; "
                          "multi-GPU sharding is not implemented (run with --gpus 1)"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2508_04917_amd import ddilu as dd
    from problems import WORKLOADS, make_workload

    torch.cuda.set_device(0)
    dd.lib()
    log(f"generating {args.workload}")
    p = make_workload(args.workload)
    sub = (0, 0, 0) if args.sub == "auto" else tuple(int(v) for v in args.sub.split(","))
    dev = "cuda:0"
    ptr_d = torch.as_tensor(p.brow_ptr, device=dev)
    col_d = torch.as_tensor(p.bcol, device=dev)
    val_d = torch.as_tensor(p.val.reshape(-1), device=dev)
    b_d = torch.as_tensor(p.b, device=dev)
    n_cu, lds = dd.dd_device_caps()
    lic_params = None
    lic_path = os.path.join(ROOT, "paper_2508_04917_amd", "lic_params.npz")
    if os.path.exists(lic_path) and p.bs == 3:
        from paper_2508_04917_amd.lic import load_params
        lic_params = torch.as_tensor(load_params(lic_path)[0], device=dev)
    log(f"device: {n_cu} CUs, {lds} B LDS per workgroup; n={p.n} nnzb={p.nnzb}")

    if args.mode == "graph":
        graph_mode(args, p, ptr_d, col_d, val_d, dd, torch)
        return
    if args.mode == "global":
        wsub = tuple(WORKLOADS[args.workload][2] or (0, 0, 0)) if args.sub == "auto" else sub
        subs = [wsub] + ([(0, 0, 0)] if args.sub == "auto" and wsub != (0, 0, 0) else [])
        dd_vs_global(args, p, subs, ptr_d, col_d, val_d, dd, torch)
        return
    if args.mode == "kernels":
        kernels_only(args, p, sub, ptr_d, col_d, val_d, dd, torch)
        return
    if args.mode == "ablation":
        ablation(args, p, sub, ptr_d, col_d, val_d, dd, torch)
        return
    if args.mode == "rocsparse":
        rocsparse_cmp(args, p, sub, ptr_d, col_d, val_d, dd, torch)
        return
    if args.mode == "precision":
        precision_mode(args, p, sub, ptr_d, col_d, val_d, lic_params, dd, torch)
        return

    def step():
        rec = {}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = dd.dd_partition(p.nx, p.ny, p.nz, p.bs, ptr_d, col_d, val_d, sub=sub)
        dd.ilu0_factor(h, dd.DD_FP64)
        torch.cuda.synchronize()
        rec["setup_s"] = time.perf_counter() - t0
        # FP64 solve with every apply timed by an event pair (the trisolve
        # GB/s), then the same solve untimed (its wall time is the plain FP64
        # solve time)
        dd.dd_set_profiling(h, True)
        x64p, i64p = dd.bicgstab_solve(h, b_d, rtol=args.rtol, maxit=args.maxit)
        dd.dd_set_profiling(h, False)
        x64, i64 = dd.bicgstab_solve(h, b_d, rtol=args.rtol, maxit=args.maxit)
        rec["fp64_profiled"] = i64p
        rec["bytes64"] = dd.dd_get_info(h)["apply_bytes"]
        t1 = time.perf_counter()
        dd.dd_set_precision(h, dd.DD_MIXED)
        torch.cuda.synchronize()
        rec["fp32_cast_s"] = time.perf_counter() - t1
        dd.dd_set_profiling(h, True)
        xmp, imp = dd.bicgstab_solve(h, b_d, rtol=args.rtol, maxit=args.maxit)
        dd.dd_set_profiling(h, False)
        xm, im = dd.bicgstab_solve(h, b_d, rtol=args.rtol, maxit=args.maxit)
        dd.dd_set_precision(h, dd.DD_FP32)
        dd.dd_set_profiling(h, True)  # FP32 trisolves: profiled solve only
        x32, i32 = dd.bicgstab_solve(h, b_d, rtol=args.rtol, maxit=args.maxit)
        dd.dd_set_profiling(h, False)
        rec["fp64"], rec["mixed"], rec["fp32"], rec["mixed_profiled"] = i64, im, i32, imp
        rec["info"] = dd.dd_get_info(h)
        rec["bytes32"] = rec["info"]["apply_bytes"]
        nx64 = torch.linalg.norm(x64)
        rec["x_rel_diff_mixed"] = float(torch.linalg.norm(xm - x64) / nx64)
        rec["x_rel_diff_fp32"] = float(torch.linalg.norm(x32 - x64) / nx64)
        rec["learned"] = None
        if lic_params is not None:
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            dd.lic_setup(h)
            dd.lic_set_params(h, lic_params)
            torch.cuda.synchronize()
            rec["lic_setup_s"] = time.perf_counter() - t2
            dd.dd_set_precision(h, dd.DD_MIXED)
            # a failed learned solve is repeated with plain DD-ILU0 inside the
            # library (dd_set_lic_fallback, on by default); info reports it
            xl, il = dd.bicgstab_solve(h, b_d, rtol=args.rtol, maxit=args.maxit)
            if il["fallback"]:
                log("learned solve failed: the result is the plain DD-ILU0 rerun")
            rec["learned"] = il
            rec["x_rel_diff_learned"] = float(torch.linalg.norm(xl - x64) / nx64)
        h.close()
        for k in ("fp64", "mixed", "fp32"):
            if rec[k]["status"] != 0:
                log(f"WARNING: {k} solve ended with status {rec[k]['status']}")
        return rec

    # reference: a plain device copy of 1 GiB (read + write), outside the timed region
    csrc = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    cdst = torch.empty_like(csrc)
    cev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    cdst.copy_(csrc)
    cev[0].record()
    for _ in range(5):
        cdst.copy_(csrc)
    cev[1].record()
    torch.cuda.synchronize()
    copy_gbs = 2 * csrc.numel() * 8 * 5 / (cev[0].elapsed_time(cev[1]) * 1e-3) / 1e9
    del csrc, cdst
    # and a plain read of 2 GiB (a sum): the apply reads 24 bytes for every
    # byte it writes, so this is the closer ceiling
    rsrc = torch.ones(1 << 28, dtype=torch.float64, device=dev)
    for _ in range(2):
        rsrc.sum()
    cev[0].record()
    for _ in range(10):
        rsrc.sum()
    cev[1].record()
    torch.cuda.synchronize()
    read_gbs = rsrc.numel() * 8 * 10 / (cev[0].elapsed_time(cev[1]) * 1e-3) / 1e9
    del rsrc

    for w in range(args.warmup):
        log(f"warmup step {w + 1}/{args.warmup}")
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = []
    for k in range(args.steps):
        recs.append(step())
        r = recs[-1]
        log(f"step {k + 1}/{args.steps}: setup {r['setup_s']:.3f}s, FP64 {r['fp64']['iters']} it "
            f"{r['fp64']['solve_seconds']:.3f}s, mixed {r['mixed']['iters']} it {r['mixed']['solve_seconds']:.3f}s, "
            f"FP32 {r['fp32']['iters']} it {r['fp32']['solve_seconds']:.3f}s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    inf = recs[0]["info"]
    applies64 = sum(r["fp64_profiled"]["applies"] for r in recs)
    secs64 = sum(r["fp64_profiled"]["apply_seconds"] for r in recs)
    applies32 = sum(r["fp32"]["applies"] for r in recs)
    secs32 = sum(r["fp32"]["apply_seconds"] for r in recs)
    appliesm = sum(r["mixed_profiled"]["applies"] for r in recs)
    secsm = sum(r["mixed_profiled"]["apply_seconds"] for r in recs)
    bytes64, bytes32 = recs[0]["bytes64"], recs[0]["bytes32"]
    gbs64 = bytes64 * applies64 / secs64 / 1e9
    gbs32 = bytes32 * applies32 / secs32 / 1e9
    gbsm = bytes32 * appliesm / secsm / 1e9
    med = lambda xs: float(np.median(xs))
    subd = [inf["sx"], inf["sy"], inf["sz"]]

    traffic = measured_traffic(args.workload, subd)
    out = {
        "metric": METRIC,
        "value": round(gbs64, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": [p.nx, p.ny, p.nz], "bs": p.bs,
                   "block_rows": p.n, "blocks": p.nnzb, "subdomain": subd, "n_subdomains": inf["nsub"],
                   "rtol": args.rtol},
        "hbm_peak_frac": round(gbs64 / HBM_PEAK_GBS, 4),
        "trisolve": {
            "fp64": {"GB/s": round(gbs64, 1), "us_per_apply": round(1e6 * secs64 / applies64, 2),
                     "bytes_per_apply": bytes64, "hbm_peak_frac": round(gbs64 / HBM_PEAK_GBS, 4)},
            "mixed_fp32_factors_fp64_math": {"GB/s": round(gbsm, 1), "us_per_apply": round(1e6 * secsm / appliesm, 2),
                                             "bytes_per_apply": bytes32, "hbm_peak_frac": round(gbsm / HBM_PEAK_GBS, 4)},
            "fp32": {"GB/s": round(gbs32, 1), "us_per_apply": round(1e6 * secs32 / applies32, 2),
                     "bytes_per_apply": bytes32, "hbm_peak_frac": round(gbs32 / HBM_PEAK_GBS, 4)},
        },
        "bicgstab": {
            "plain_fp64": {"iters": recs[0]["fp64"]["iters"], "status": recs[0]["fp64"]["status"],
                           "solve_s": round(med([r["fp64"]["solve_seconds"] for r in recs]), 4),
                           "rel_res_true": recs[0]["fp64"]["rel_res_true"]},
            "mixed_fp32_factors": {"iters": recs[0]["mixed"]["iters"], "status": recs[0]["mixed"]["status"],
                                   "solve_s": round(med([r["mixed"]["solve_seconds"] for r in recs]), 4),
                                   "rel_res_true": recs[0]["mixed"]["rel_res_true"],
                                   "x_rel_diff_vs_fp64": recs[0]["x_rel_diff_mixed"]},
            "fp32": {"iters": recs[0]["fp32"]["iters"], "status": recs[0]["fp32"]["status"],
                     "solve_s_with_apply_timing": round(med([r["fp32"]["solve_seconds"] for r in recs]), 4),
                     "restarts": recs[0]["fp32"]["restarts"],
                     "rel_res_true": recs[0]["fp32"]["rel_res_true"],
                     "x_rel_diff_vs_fp64": recs[0]["x_rel_diff_fp32"]},
            "setup_s": round(med([r["setup_s"] for r in recs]), 4),
            "learned_mixed": None if recs[0]["learned"] is None else {
                "iters": recs[0]["learned"]["iters"], "status": recs[0]["learned"]["status"],
                "solve_s": round(med([r["learned"]["solve_seconds"] for r in recs]), 4),
                "lic_setup_s": round(med([r["lic_setup_s"] for r in recs]), 4),
                "rel_res_true": recs[0]["learned"]["rel_res_true"],
                "x_rel_diff_vs_fp64": recs[0]["x_rel_diff_learned"],
                "fallback": bool(recs[0]["learned"]["fallback"])},
        },
        "roofline": {"bound": "hbm", "achieved": round(gbs64, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs64 / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "k_dd_apply_slots<3, double, double, 1024, 3, 2, false, false>",
                     "bytes_per_launch": bytes64, "copy_GBs": round(copy_gbs, 1),
                     "frac_of_copy": round(gbs64 / copy_gbs, 4), "read_GBs": round(read_gbs, 1),
                     "frac_of_read": round(gbs64 / read_gbs, 4)},
        "cpu_baseline": None,
    }

    if args.extra:
        out["workloads"] = {}
        for wname, override in (("aniso160_bsr3", {}), ("lognormal128_eval", {})):
            out["workloads"][wname] = compare_workload(args, wname, override, lic_params, dd, torch, np)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, p, tuple(subd), bytes64, np, gpu_iters=recs[0]["fp64"]["iters"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
