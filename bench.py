"""Benchmark: online random-walker interaction on the 512 x 512 workload (one MI355X).

A step is one pass of the online hot path over one batch of synthetic input:
  graph rebuild from J (beta = 90), restore of the precomputed basis,
  solve with the seed-driven choice of m (eps = 0.1),
  then three cumulative edits (beta -> 150; a 32 x 32 block of edges scaled by 0.1; 500 random
  edges removed), each followed by a Rayleigh-Ritz eigenvector update and a new solve.
That is 4 RW solves and 3 eigenvector updates per step; value = RW solves per second including
the updates between them.  The offline eigenpairs (m = 200, tol 1e-5) are computed once before the
timed region.  Outside the timed region the script also measures, per edit, the refined update
(Rayleigh-Ritz + filtered iterations to tol) against a cold recompute at the same tol and m, and the
stencil operator's HBM throughput on an N x (m + guard) block.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-compare] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-compare", action="store_true", help="skip the update-vs-recompute comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-eigsh", action="store_true",
                    help="also time the oracle's eigsh recompute of the 512x512 basis (minutes of CPU time)")
    ap.add_argument("--spmm-reps", type=int, default=20)
    ap.add_argument("--traffic-probe", action="store_true",
                    help="only launch the stencil block and a plain copy of the same block (for HBM counters)")
    ap.add_argument("--workload", default="interactive512",
                    choices=["interactive512", "small64", "volume128", "batch64", "grad96", "prior512", "bank512",
                             "agg512", "rwir96"],
                    help="interactive512 (default, the headline line); the others measure the remaining "
                         "configurations and print their own line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1 (sharding across GPUs is "
                                   "not implemented)"}))
        sys.exit(2)

    import torch
    import paper_1607_04174_amd as rw
    import rwsynth

    dev = torch.device("cuda", 0)
    w = rwsynth.CFG2
    if args.traffic_probe:
        traffic_probe(rw, rwsynth, torch, rwsynth.CFG3 if args.workload == "volume128" else w, dev)
        return
    if args.workload != "interactive512":
        line = MODES[args.workload](args, rw, rwsynth, torch, dev)
        print(json.dumps(line), flush=True)
        return
    J, rid = rwsynth.phantom(w, 0)
    node, lab = rwsynth.seeds(w, rid, 0)
    edits = rwsynth.cfg2_edits(w, 0)
    Jd = torch.as_tensor(J, device=dev)
    dt = torch.float32
    tol = 1e-5
    log(f"workload {w.name}: N={w.N} m={w.m} C={w.C} S={node.size}")

    # ---- offline: eigenpairs at beta = 90 ----
    g = rw.Graph(Jd, w.dims, w.conn, w.beta, dtype=dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Q0, lam0, einfo = rw.precompute_eig(g, w.m, tol=tol, max_iter=400)
    torch.cuda.synchronize()
    t_pre = time.perf_counter() - t0
    log(f"precompute: {t_pre:.2f}s iters={einfo['iters']} res={einfo['max_residual']:.2e} "
        f"spmm_cols={einfo['spmm_columns']}")

    Q = torch.empty_like(Q0)
    lam = torch.empty_like(lam0)
    ws = rw.SolveWorkspace()
    U = torch.empty((w.C, w.N), dtype=dt, device=dev)

    def step():
        gs = rw.Graph(Jd, w.dims, w.conn, w.beta, dtype=dt)
        Q.copy_(Q0)
        lam.copy_(lam0)
        ms = []
        _, inf = rw.solve_seeds(gs, Q, lam, node, lab, w.C, eps=0.1, U=U, workspace=ws)
        ms.append((inf["m_used"], inf["eig_probes"]))
        for e in edits:
            rw.update_eig(gs, [e], Q, lam, mode=rw.RW_UPDATE_RR, tol=tol)
            _, inf = rw.solve_seeds(gs, Q, lam, node, lab, w.C, eps=0.1, U=U, workspace=ws)
            ms.append((inf["m_used"], inf["eig_probes"]))
        return ms

    for _ in range(args.warmup):
        m_used = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        m_used = step()
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    ms_per_step = 1000.0 * T / args.steps
    solves_per_step = 1 + len(edits)
    value = solves_per_step * args.steps / T
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step, {value:.2f} solves/s, m_used={m_used}")

    # ---- stencil operator throughput (dominant HBM kernel), HIP events on the launch stream ----
    # Timing protocol: before every timed launch (outside the events) 1.25 GiB are written and then
    # 512 MiB of another buffer are read, so the operands start in HBM, not in the 256 MB Infinity Cache
    # or the L2s, and the cache holds clean lines (the flush's own dirty lines are written back during the
    # read sweep, not during the timed launch).  The unflushed figure (launches back to back on the same
    # block) is reported beside it, and a plain device copy of the block under the same protocol gives the
    # practical peak.
    nb = stencil_block_cols(w)
    ndir = 4
    es = 4
    flush_w = torch.empty(5 << 28, dtype=torch.uint8, device=dev)    # 1.25 GiB written
    flush_r = torch.ones(1 << 27, dtype=torch.float32, device=dev)    # 512 MiB read
    stream = torch.cuda.current_stream()

    def do_flush(k):
        flush_w.fill_(k & 0xFF)
        return flush_r.sum()

    def event_us(fn, flushed):
        ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.spmm_reps)]
        ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.spmm_reps)]
        for k in range(args.spmm_reps):
            if flushed:
                do_flush(k)
            ev0[k].record(stream)
            fn(k)
            ev1[k].record(stream)
        torch.cuda.synchronize()
        return 1e3 * float(np.mean([a.elapsed_time(b) for a, b in zip(ev0, ev1)]))

    def stencil_us(cols, flushed):
        """(dispatch us, bracketed us) per launch: the kernel's own start and end recorded by the launch
        (the interval a kernel trace reports), and the stream events recorded before and after it."""
        X = torch.randn((cols, w.N), dtype=dt, device=dev)
        Y = torch.empty_like(X)
        for _ in range(3):
            rw.apply_laplacian(g, X, Y)
        d0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.spmm_reps)]
        d1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.spmm_reps)]
        br = event_us(lambda k: rw.apply_laplacian_timed(g, X, Y, d0[k], d1[k]), flushed)
        return 1e3 * float(np.mean([a.elapsed_time(b) for a, b in zip(d0, d1)])), br

    def copy_us():
        X = torch.randn((nb, w.N), dtype=dt, device=dev)
        Y = torch.empty_like(X)
        Y.copy_(X)
        return event_us(lambda k: Y.copy_(X), True)

    def stencil_bytes(cols):
        return w.N * (2 * es * cols + es * (ndir + 1))       # read X, write Y, coefficients + diagonal

    spmm_us, spmm_us_br = stencil_us(nb, True)
    spmm_us_warm, _ = stencil_us(nb, False)
    step_cols = w.m - 1                                        # the update step's operator block
    step_us, _ = stencil_us(step_cols, True)
    spmm_bytes = stencil_bytes(nb)
    cp_us = copy_us()
    spmm_gbs = spmm_bytes / (spmm_us * 1e-6) / 1e9
    spmm_gbs_warm = spmm_bytes / (spmm_us_warm * 1e-6) / 1e9
    spmm_gbs_br = spmm_bytes / (spmm_us_br * 1e-6) / 1e9
    step_gbs = stencil_bytes(step_cols) / (step_us * 1e-6) / 1e9
    copy_gbs = 2 * es * nb * w.N / (cp_us * 1e-6) / 1e9
    del flush_w, flush_r
    log(f"stencil N x {nb} fp32: {spmm_us:.1f} us/launch flushed ({spmm_gbs:.0f} GB/s; {spmm_us_br:.1f} us between "
        f"stream events around it), {spmm_us_warm:.1f} us "
        f"back to back ({spmm_gbs_warm:.0f} GB/s); N x {step_cols}: {step_us:.1f} us ({step_gbs:.0f} GB/s); "
        f"copy of the block {cp_us:.1f} us ({copy_gbs:.0f} GB/s)")

    # ---- update vs recompute at equal accuracy (same tol, same m), medians of 3 runs each ----
    # The edits are cumulative: edit i is applied to the graph after edits 0..i-1, starting from the pairs the
    # previous update produced.  Each repetition rebuilds that starting state untimed.
    compare = None
    if not args.no_compare:
        reps = 3
        Qs, lams = Q0.clone(), lam0.clone()
        rows = []
        for i, e in enumerate(edits):
            t_upd, t_rec = [], []
            for r in range(reps):
                gs = rw.Graph(Jd, w.dims, w.conn, w.beta, dtype=dt)
                if i > 0:
                    rw.edit_graph(gs, edits[:i])
                Qc, lamc = Qs.clone(), lams.clone()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ui = rw.update_eig(gs, [e], Qc, lamc, mode=rw.RW_UPDATE_RR_REFINE, tol=tol, max_iter=400)
                torch.cuda.synchronize()
                t_upd.append(time.perf_counter() - t0)
                t0 = time.perf_counter()
                Qr, lamr, ri = rw.precompute_eig(gs, w.m, tol=tol, max_iter=400, seed=7)
                torch.cuda.synchronize()
                t_rec.append(time.perf_counter() - t0)
            Qs, lams = Qc, lamc
            rows.append({"edit": e.kind, "update_s": round(float(np.median(t_upd)), 4),
                         "recompute_s": round(float(np.median(t_rec)), 4), "reps": reps,
                         "update_iters": ui["iters"], "recompute_iters": ri["iters"],
                         "update_spmm_columns": ui["spmm_columns"], "recompute_spmm_columns": ri["spmm_columns"],
                         "update_res": ui["max_residual"], "recompute_res": ri["max_residual"],
                         "max_dlambda": float((lamc - lamr).abs().max())})
            log(f"edit {e.kind}: update {np.median(t_upd):.3f}s vs recompute {np.median(t_rec):.3f}s "
                f"(medians of {reps})")
        compare = rows

    # ---- CPU oracle baseline on a bounded sample ----
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, J, node, lab, edits, Q0, lam0, solves_per_step)
        if args.cpu_eigsh:
            cpu["recompute"] = cpu_recompute_eigsh(w, J, w.m)

    out = {
        "metric": "RW solves/s + eigvec-update vs recompute time at fixed error; SpMV HBM GB/s",
        "value": round(value, 3),
        "unit": "RW solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (stencil, Q, U, Gram chunks) + f64 (Gram sums, Rayleigh-Ritz, seed system)",
        "data": "synthetic",
        "config": {"workload": "2D 512x512 8-connected phantom, beta 90, m=200, C=3, 50 seeds/label; "
                               "per step 4 solves (eps=0.1) + 3 edits with Rayleigh-Ritz updates",
                   "N": w.N, "m": w.m, "C": w.C, "S": int(node.size), "m_used": [a for a, _ in m_used],
                   "eig_probes": [b for _, b in m_used]},
        "precompute_s": round(t_pre, 3),
        "spmv_gbs": round(spmm_gbs, 1),
        "update_vs_recompute": compare,
        "roofline": {"kernel": "k_stencil_strip<float,4,8,plain,buffer,WX=2,PF=2> (N x %d block)" % nb, "bound": "hbm",
                     "achieved": round(spmm_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(spmm_gbs / PEAK_HBM_GBS, 4), "traffic": stencil_traffic(nb, w.N),
                     "bytes_per_launch": spmm_bytes, "us_per_launch": round(spmm_us, 2),
                     "timing": "HIP events recorded by each launch at the kernel's own start and end "
                               "(hipExtLaunchKernel), on the launch stream; before each launch 1.25 GiB written "
                               "then 512 MiB of another buffer read",
                     "stream_events": {"achieved": round(spmm_gbs_br, 1), "us_per_launch": round(spmm_us_br, 2),
                                       "note": "events recorded on the stream before and after the launch"},
                     "copy_same_protocol": {"achieved": round(copy_gbs, 1), "us_per_launch": round(cp_us, 2),
                                            "frac": round(copy_gbs / PEAK_HBM_GBS, 4),
                                            "note": "torch copy_ of the block between stream events"},
                     "unflushed": {"achieved": round(spmm_gbs_warm, 1), "us_per_launch": round(spmm_us_warm, 2)},
                     "in_step_shape": {"cols": step_cols, "achieved": round(step_gbs, 1),
                                       "us_per_launch": round(step_us, 2),
                                       "frac": round(step_gbs / PEAK_HBM_GBS, 4)}},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def stencil_block_cols(w):
    """Columns of the eigensolver's working block for m pairs (m - 1 + guard)."""
    return w.m - 1 + max(8, (w.m + 9) // 10)


def traffic_probe(rw, rwsynth, torch, w, dev):
    """Five launches of the stencil on the N x nb block, then five plain device copies of the same block
    (torch's copy kernel), for reading FETCH_SIZE / WRITE_SIZE per dispatch under the profiler."""
    J, _ = rwsynth.phantom(w, 0)
    g = rw.Graph(torch.as_tensor(J, device=dev), w.dims, w.conn, w.beta, dtype=torch.float32)
    nb = stencil_block_cols(w)
    X = torch.randn((nb, w.N), dtype=torch.float32, device=dev)
    Y = torch.empty_like(X)
    for _ in range(5):
        rw.apply_laplacian(g, X, Y)
    torch.cuda.synchronize()
    for _ in range(5):
        Y.copy_(X)
    torch.cuda.synchronize()
    log(f"traffic probe: stencil and copy of {nb} x {w.N} fp32 ({nb * w.N * 4} bytes per block), 5 launches each")


def stencil_traffic(nb, N):
    """HBM bytes per stencil launch from the committed counter summary, if it was taken on the current
    kernel source (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "stencil_traffic.json")
    src = os.path.join(ROOT, "paper_1607_04174_amd", "csrc", "stencil.hip")
    try:
        with open(path) as f:
            rec = json.load(f)
        with open(src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if rec.get("stencil_source_sha256") != sha or rec.get("cols") != nb or rec.get("N") != N:
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(w, J, node, lab, edits, Q0, lam0, solves_per_step):
    """The oracle (FP64 numpy/scipy) on one solve and one update of the same workload, scaled to a step."""
    import torch
    from oracle.choose_m import choose_m
    from oracle.fast_rw import fast_rw_coeffs
    from oracle.graph import Graph as OGraph
    from oracle.update import rayleigh_ritz
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    Q = Q0.to(torch.float64).cpu().numpy().T
    lam = lam0.cpu().numpy()
    n_upd = solves_per_step - 1

    def sample():
        og = OGraph(J, w.dims, w.conn, w.beta)
        t0 = time.perf_counter()
        m, _, _ = choose_m(og, Q, node, lab, w.C, eps=0.1)
        fast_rw_coeffs(og, Q, lam, node, lab, w.C, m=m)
        t_solve = time.perf_counter() - t0
        og.apply_edit(edits[0])
        t0 = time.perf_counter()
        rayleigh_ritz(og, Q)
        return t_solve, time.perf_counter() - t0

    t_solve, t_upd = sample()
    step_s = solves_per_step * t_solve + n_upd * t_upd
    log(f"cpu oracle: solve {t_solve:.2f}s, update {t_upd:.2f}s -> {solves_per_step / step_s:.4f} solves/s")
    single = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            s1, u1 = sample()
        single = {"value": round(solves_per_step / (solves_per_step * s1 + n_upd * u1), 5), "cores": 1,
                  "solve_s": round(s1, 3), "update_s": round(u1, 3)}
        log(f"cpu oracle, one thread: solve {s1:.2f}s, update {u1:.2f}s")
    except ImportError:
        pass
    return {"value": round(solves_per_step / step_s, 5), "unit": "RW solves/s", "cores": int(cores),
            "kind": "oracle",
            "sample": "one solve (choice of m by linear scan, bordered system, coefficients) and one "
                      "Rayleigh-Ritz update (beta edit) of the 512x512 workload, FP64, scaled to a step of "
                      f"{solves_per_step} solves + {n_upd} updates",
            "solve_s": round(t_solve, 3), "update_s": round(t_upd, 3), "single_thread": single}


def cpu_recompute_eigsh(w, J, m, tol=1e-5):
    """The oracle's recompute of the m smallest eigenpairs of the 512x512 operator by scipy's eigsh
    (shift-invert about a point below the spectrum), for the update-vs-recompute comparison on the CPU."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    from oracle.graph import Graph as OGraph
    og = OGraph(J, w.dims, w.conn, w.beta)
    M = og.M().tocsc()
    t0 = time.perf_counter()
    vals, _ = spla.eigsh(M, k=m, sigma=-1e-3, which="LM", tol=tol)
    t = time.perf_counter() - t0
    log(f"cpu oracle eigsh: {m} pairs in {t:.1f}s")
    return {"eigsh_recompute_s": round(t, 2), "pairs": m, "tol": tol, "lambda_max": float(vals.max())}


# ---------------------------------------------------------------------------------------------
# the other workloads (one JSON line each; the default run prints only the interactive512 line)
# ---------------------------------------------------------------------------------------------
def _sync_time(torch, fn, reps):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, out


def _cores():
    try:
        from threadpoolctl import threadpool_info
        return max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        return os.cpu_count()


def _line(metric, value, unit, args, ms_per_step, dtype, config, **extra):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}
    out.update(extra)
    return out


def run_small64(args, rw, rwsynth, torch, dev):
    """64 x 64, 4-connected, FP64: exact RW by CG and the eigenbasis solve (m = 50), both against the oracle."""
    w = rwsynth.CFG1
    J, rid = rwsynth.phantom(w, 0)
    node, lab = rwsynth.seeds(w, rid, 0)
    Jd = torch.as_tensor(J, device=dev)
    g = rw.Graph(Jd, w.dims, w.conn, w.beta, dtype=torch.float64)
    t_pre, (Q, lam, einfo) = _sync_time(torch, lambda: rw.precompute_eig(g, w.m, tol=1e-10, max_iter=400), 1)
    ws = rw.SolveWorkspace()
    for _ in range(args.warmup):
        rw.cg_solve(g, node, lab, w.C, tol=1e-12)
        rw.solve_seeds(g, Q, lam, node, lab, w.C, workspace=ws)
    t_cg, (Ucg, cinfo) = _sync_time(torch, lambda: rw.cg_solve(g, node, lab, w.C, tol=1e-12), args.steps)
    t_eig, (Ue, _) = _sync_time(torch, lambda: rw.solve_seeds(g, Q, lam, node, lab, w.C, workspace=ws), args.steps)
    log(f"small64: CG {t_cg * 1e3:.2f} ms/solve ({cinfo['iters']} it), eigenbasis {t_eig * 1e3:.3f} ms/solve")
    parity = None
    cpu = None
    if not args.no_cpu:
        from oracle.exact_rw import exact_rw
        from oracle.fast_rw import fast_rw
        from oracle.graph import Graph as OGraph
        og = OGraph(J, w.dims, w.conn, w.beta)
        t0 = time.perf_counter()
        Ud = exact_rw(og, node, lab, w.C, method="cg", tol=1e-12)
        t_ocg = time.perf_counter() - t0
        Qn, ln = Q.cpu().numpy().T, lam.cpu().numpy()
        exact = bool(np.min(np.abs(ln[1:])) < 1e-6)
        t0 = time.perf_counter()
        Uf = fast_rw(og, Qn, ln, node, lab, w.C, exact=exact)
        t_ofast = time.perf_counter() - t0
        parity = {"cg_vs_oracle_maxabs": float(np.abs(Ucg.cpu().numpy().T - Ud).max()),
                  "eig_vs_oracle_same_basis_maxabs": float(np.abs(Ue.cpu().numpy().T - Uf).max()),
                  "eig_truncation_vs_exact_maxabs": float(np.abs(Ue.cpu().numpy().T - Ud).max())}
        cpu = {"value": round(1.0 / t_ofast, 4), "unit": "RW solves/s", "cores": int(_cores()), "kind": "oracle",
               "sample": "one eigenbasis solve (bordered system, FP64%s) of the 64x64 workload; the oracle's "
                         "CG exact solve took %.3f s" % (", exact rational arithmetic" if exact else "", t_ocg)}
    return _line("RW solves/s (eigenbasis, m = 50) and exact CG solves/s", round(1.0 / t_eig, 2), "RW solves/s",
                 args, t_eig * 1e3, "f64",
                 {"workload": "2D 64x64 4-connected phantom, beta 90, m=50, C=2, 20 seeds/label, FP64",
                  "N": w.N, "m": w.m, "C": w.C, "S": int(node.size)},
                 cg_solves_per_s=round(1.0 / t_cg, 2), cg_iters=cinfo["iters"], precompute_s=round(t_pre, 3),
                 eig_max_residual=einfo["max_residual"], parity=parity, cpu_baseline=cpu)


def _window_sines(torch, Qa, lama, Qb, lamb, delta):
    """Per column i of Qa: sin of its angle to span{Qb_j : |lamb_j - lama_i| <= delta} (Davis-Kahan: at
    most ||r_i|| / delta).  A window that reaches the last stored pair may need pairs beyond the cut;
    those columns are flagged.  FP64 on the device (analysis only)."""
    m = Qa.shape[0]
    la, lb = lama.double().cpu().numpy(), lamb.double().cpu().numpy()
    sines = np.zeros(m)
    crossing = np.zeros(m, dtype=bool)
    for i in range(m):
        sel = np.abs(lb - la[i]) <= delta
        crossing[i] = la[i] + delta >= lb[-1]
        q = Qa[i].double()
        Qw = Qb[torch.as_tensor(np.flatnonzero(sel), device=Qb.device)].double()
        r = q - (Qw @ q) @ Qw                            # component outside the window's span
        sines[i] = (r.norm() / q.norm()).item()
    return sines, crossing


def run_volume128(args, rw, rwsynth, torch, dev):
    """128^3, 6-connected, mixed precision: FP32 eigensolver and stencil, BF16 Q (pair form) on the matrix
    cores, FP64 Gram / Cholesky-QR / Rayleigh-Ritz / seed system; errors against the FP64 path for every
    eigenpair and every map; solve throughput with the BF16 pair-form basis (the plain BF16 copy beside it)."""
    w = rwsynth.CFG3
    J, rid = rwsynth.phantom(w, 0)
    node, lab = rwsynth.seeds(w, rid, 0)
    Jd = torch.as_tensor(J, device=dev)
    g32 = rw.Graph(Jd, w.dims, w.conn, w.beta, dtype=torch.float32)
    t32, (Q32, lam32, i32) = _sync_time(torch, lambda: rw.precompute_eig(g32, w.m, tol=1e-6, max_iter=400), 1)
    log(f"volume128: FP32 precompute {t32:.2f}s it={i32['iters']} res={i32['max_residual']:.2e}")
    g64 = rw.Graph(Jd, w.dims, w.conn, w.beta, dtype=torch.float64)
    t64, (Q64, lam64, i64) = _sync_time(torch, lambda: rw.precompute_eig(g64, w.m, tol=1e-10, max_iter=800), 1)
    log(f"volume128: FP64 precompute {t64:.2f}s it={i64['iters']} res={i64['max_residual']:.2e}")
    dlam = (lam32 - lam64).abs().cpu().numpy()
    sines, crossing = _window_sines(torch, Q32, lam32, Q64, lam64, delta=1e-4)
    Qb = rw.to_pair(Q32)
    Q64b = rw.to_pair(Q64)
    Qplain = rw.convert_block(Q32, torch.bfloat16)
    Q64plain = rw.convert_block(Q64, torch.bfloat16)
    ws = rw.SolveWorkspace()
    ev = lam64.cpu().numpy()
    gaps = np.diff(ev)
    mcut = int(w.m // 2 + np.argmax(gaps[w.m // 2 - 1:]) + 1)      # largest gap in the upper half
    err = {}
    for tag, mm in (("m", w.m), ("gap_cut", mcut)):
        U64, _ = rw.solve_seeds(g64, Q64, lam64, node, lab, w.C, m_avail=mm, workspace=ws)
        U32s, _ = rw.solve_seeds(g32, Q64.float(), lam64, node, lab, w.C, m_avail=mm, workspace=ws)
        U16s, _ = rw.solve_seeds(g32, Q64b, lam64, node, lab, w.C, m_avail=mm, workspace=ws)
        U32, _ = rw.solve_seeds(g32, Q32, lam32, node, lab, w.C, m_avail=mm, workspace=ws)
        U16, _ = rw.solve_seeds(g32, Qb, lam32, node, lab, w.C, m_avail=mm, workspace=ws)
        Upl, _ = rw.solve_seeds(g32, Qplain, lam32, node, lab, w.C, m_avail=mm, workspace=ws)
        Upls, _ = rw.solve_seeds(g32, Q64plain, lam64, node, lab, w.C, m_avail=mm, workspace=ws)
        err[tag] = {"m": mm,
                    "same_basis_fp32_maxabs": float((U32s.double() - U64).abs().max()),
                    "same_basis_bf16_pair_maxabs": float((U16s.double() - U64).abs().max()),
                    "same_basis_bf16_plain_maxabs": float((Upls.double() - U64).abs().max()),
                    "end_to_end_fp32_maxabs": float((U32.double() - U64).abs().max()),
                    "end_to_end_bf16_pair_maxabs": float((U16.double() - U64).abs().max()),
                    "end_to_end_bf16_plain_maxabs": float((Upl.double() - U64).abs().max()),
                    "per_map_end_to_end_bf16_maxabs": [float((U16[c].double() - U64[c]).abs().max())
                                                       for c in range(w.C)]}
    ok = ~crossing
    err["eig_abs_dlambda_max"] = float(dlam.max())
    err["eig_abs_dlambda"] = [float(x) for x in dlam]
    err["eig_sin_angle_max_inside"] = float(sines[ok].max()) if ok.any() else None
    err["eig_pairs_window_crosses_cut"] = int(crossing.sum())
    err["eig_sin_angle"] = [float(x) for x in sines]
    U16 = torch.empty((w.C, w.N), dtype=torch.float32, device=dev)
    U32 = torch.empty_like(U16)
    log(f"volume128: errors vs FP64 path: {err['m']} {err['gap_cut']} dlambda {err['eig_abs_dlambda_max']:.2e} "
        f"sin {err['eig_sin_angle_max_inside']} (crossing {err['eig_pairs_window_crosses_cut']})")
    for _ in range(args.warmup):
        rw.solve_seeds(g32, Qb, lam32, node, lab, w.C, U=U16, workspace=ws)
    t16, _ = _sync_time(torch, lambda: rw.solve_seeds(g32, Qb, lam32, node, lab, w.C, U=U16, workspace=ws),
                        args.steps)
    t32s, _ = _sync_time(torch, lambda: rw.solve_seeds(g32, Q32, lam32, node, lab, w.C, U=U32, workspace=ws),
                         args.steps)
    tpl, _ = _sync_time(torch, lambda: rw.solve_seeds(g32, Qplain, lam32, node, lab, w.C, U=U32, workspace=ws),
                        args.steps)
    # reconstruction kernel alone (matrix cores, BF16 Q): HIP events on the launch stream
    stream = torch.cuda.current_stream()
    reps = 10
    e0 = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
    e1 = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
    for k in range(reps):
        e0[k].record(stream)
        rw.solve_seeds(g32, Qb, lam32, node, lab, w.C, U=U16, workspace=ws)
        e1[k].record(stream)
    torch.cuda.synchronize()
    solve_ms = float(np.mean([a.elapsed_time(b) for a, b in zip(e0, e1)]))
    log(f"volume128: solve BF16 pair {t16 * 1e3:.2f} ms, plain BF16 {tpl * 1e3:.2f} ms, FP32 {t32s * 1e3:.2f} ms")
    return _line("RW solves/s (BF16 pair-form eigenbasis on the matrix cores) with errors against the FP64 path",
                 round(1.0 / t16, 2), "RW solves/s", args, t16 * 1e3,
                 "f32 stencil/blocks + bf16 pair-form Q (MFMA, f32 accumulation) + f64 Gram/RR/seed system",
                 {"workload": "3D 128^3 6-connected phantom (8 ellipsoids, uniform intensities, sigma 0.03), "
                              "beta 120, m=100, C=4, 200 seeds/label", "N": w.N, "m": w.m, "C": w.C,
                  "S": int(node.size)},
                 fp32_solves_per_s=round(1.0 / t32s, 2), plain_bf16_solves_per_s=round(1.0 / tpl, 2),
                 gap_cut_m=mcut, precompute_fp32_s=round(t32, 2),
                 precompute_fp64_s=round(t64, 2), fp32_max_residual=i32["max_residual"],
                 fp64_max_residual=i64["max_residual"], errors=err, solve_event_ms=round(solve_ms, 3))


def run_batch64(args, rw, rwsynth, torch, dev):
    """64 uneven 2D images x 8 seed-set rounds; one HIP-graph replay per round."""
    imgs = rwsynth.cfg4_images(64, 0)
    rounds = 8
    images, rid_of = [], []
    t0 = time.perf_counter()
    for i, w in enumerate(imgs):
        J, rid = rwsynth.phantom(w, 0)
        g = rw.Graph(torch.as_tensor(J, device=dev), w.dims, w.conn, w.beta, dtype=torch.float32)
        Q, lam, _ = rw.precompute_eig(g, w.m, tol=1e-5, max_iter=400)
        rnds = [rwsynth.cfg4_round(w, rid, r, 0) for r in range(rounds)]
        images.append({"graph": g, "Q": Q, "lam": lam, "rounds": rnds, "C_cap": 4,
                       "S_cap": max(len(x[1]) for x in rnds)})
    torch.cuda.synchronize()
    t_pre = time.perf_counter() - t0
    elems = sum(im["graph"].N * im["Q"].shape[0] for im in images)
    log(f"batch64: precompute of 64 bases {t_pre:.1f}s, sum N_i m_i = {elems:.3e}")
    bs = rw.BatchSolver(images, use_graph=True)
    info = bs.info()
    # round r of the timed region uses interaction r mod 8; the seeds of each round are set (host
    # validation + upload) inside the timed region, as an interactive session would
    for r in range(args.warmup):
        bs.set_seeds([im["rounds"][r % rounds] for im in images])
        bs.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(args.steps * rounds):
        bs.set_seeds([im["rounds"][r % rounds] for im in images])
        bs.run()
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    per_round = T / (args.steps * rounds)
    pivot = bs.status()
    # one round's replay alone (seeds already resident): HIP events on the replay stream
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(5):
        bs.run()
    e1.record(stream)
    torch.cuda.synchronize()
    replay_ms = e0.elapsed_time(e1) / 5
    qbytes = sum(im["graph"].N * im["Q"].shape[0] * 4 for im in images)
    ubytes = sum(im["graph"].N * int(im["rounds"][0][0]) * 4 for im in images)
    gbs = (qbytes + ubytes) / (replay_ms * 1e-3) / 1e9
    log(f"batch64: {per_round * 1e3:.2f} ms/round incl. seed upload, replay {replay_ms:.2f} ms, "
        f"{64 / per_round:.0f} image-interactions/s, tile {info}")
    return _line("batched interactions/s (images x seed-set rounds per second)", round(64 / per_round, 1),
                 "image-interactions/s", args, per_round * 1e3 * rounds,
                 "f32 Q and U + f64 seed systems",
                 {"workload": "64 2D phantoms, sides uniform in [128, 768], 4-connected, beta 90, m in {50, 100, "
                              "200}, 8 seed-set rounds (C 2-4, 10-100 seeds/label), one HIP-graph replay per round",
                  "images": 64, "rounds_per_step": rounds, "sum_N_m": int(elems)},
                 ms_per_round=round(per_round * 1e3, 3), replay_ms=round(replay_ms, 3), precompute_s=round(t_pre, 1),
                 autotune=info, min_pivot=pivot,
                 roofline={"kernel": "k_b_reconstruct (whole round)", "bound": "hbm", "achieved": round(gbs, 1),
                           "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
                           "traffic": None, "bytes_per_launch": qbytes + ubytes,
                           "note": "Q read + U write per round over the replay's duration (all kernels)"})


def run_grad96(args, rw, rwsynth, torch, dev):
    """96^3 exact RW (FP64 CG warm-started from the eigenbasis) forward + adjoint backward; central finite
    differences on sampled entries."""
    w = rwsynth.CFG5
    J, rid = rwsynth.phantom(w, 0)
    node, lab = rwsynth.seeds(w, rid, 0)
    gt = rwsynth.label_map(rid, w.C)
    Jd = torch.as_tensor(J, device=dev, dtype=torch.float64)
    g = rw.Graph(Jd, w.dims, w.conn, w.beta, dtype=torch.float64)
    t_pre, (Q, lam, _) = _sync_time(torch, lambda: rw.precompute_eig(g, w.m, tol=1e-8, max_iter=600), 1)
    scale = torch.ones((3, w.N), dtype=torch.float64, device=dev)
    mask = torch.ones(w.N, dtype=torch.bool, device=dev)
    mask[torch.as_tensor(node, device=dev)] = False
    y = torch.as_tensor(gt, device=dev, dtype=torch.long)

    def loss_of(U):
        p = U.gather(0, y[None, :])[0]
        return -(torch.log(torch.clamp(p[mask], min=1e-12))).mean()

    def fwd_bwd():
        Jt = Jd.clone().requires_grad_(True)
        bt = torch.tensor(w.beta, dtype=torch.float64, device=dev, requires_grad=True)
        st = scale.clone().requires_grad_(True)
        U = rw.random_walker(Jt, bt, st, w.dims, w.conn, node, lab, w.C, Q=Q, lam=lam, tol=1e-12)
        L = loss_of(U)
        L.backward()
        return float(L), Jt.grad, bt.grad, st.grad

    for _ in range(args.warmup):
        fwd_bwd()
    t_fb, (L0, dJ, db, ds) = _sync_time(torch, fwd_bwd, args.steps)

    def fwd(J_=None, beta=w.beta, s=scale):
        with torch.no_grad():
            U = rw.random_walker(Jd if J_ is None else J_, torch.tensor(beta, dtype=torch.float64), s, w.dims,
                                 w.conn, node, lab, w.C, Q=Q, lam=lam, tol=1e-13)
            return float(loss_of(U))

    t_f, _ = _sync_time(torch, fwd, 1)
    h = 1e-6
    rng = np.random.default_rng(5)
    checks = []
    for i in rng.choice(w.N, 3, replace=False):
        Jp, Jm = Jd.clone(), Jd.clone()
        Jp[int(i)] += h
        Jm[int(i)] -= h
        fd = (fwd(J_=Jp) - fwd(J_=Jm)) / (2 * h)
        checks.append({"param": f"J[{int(i)}]", "fd": fd, "adjoint": float(dJ[int(i)])})
    fd = (fwd(beta=w.beta + h) - fwd(beta=w.beta - h)) / (2 * h)
    checks.append({"param": "beta", "fd": fd, "adjoint": float(db)})
    for e in rng.choice(w.N - 20000, 2, replace=False):
        sp, sm = scale.clone(), scale.clone()
        sp[0, int(e)] += h
        sm[0, int(e)] -= h
        fd = (fwd(s=sp) - fwd(s=sm)) / (2 * h)
        checks.append({"param": f"s[+x, {int(e)}]", "fd": fd, "adjoint": float(ds[0, int(e)])})
    worst = max(abs(c["fd"] - c["adjoint"]) / max(1.0, abs(c["fd"])) for c in checks)
    log(f"grad96: forward+backward {t_fb:.3f}s (forward alone {t_f:.3f}s), loss {L0:.6f}, FD worst rel {worst:.2e}")
    return _line("forward + backward (exact RW, adjoint gradients w.r.t. J, beta and per-edge scales) per second",
                 round(1.0 / t_fb, 3), "forward+backward/s", args, t_fb * 1e3, "f64",
                 {"workload": "3D 96^3 6-connected phantom (5 ellipsoids, sigma 0.05), beta 120, m=80 (warm start), "
                              "C=2, 100 seeds/label, cross-entropy vs the ground-truth mask", "N": w.N,
                  "S": int(node.size)},
                 forward_s=round(t_f, 4), precompute_s=round(t_pre, 2), loss=L0, fd_checks=checks,
                 fd_worst_rel=worst)


def run_prior512(args, rw, rwsynth, torch, dev):
    """512 x 512, 8-connected, FP32 graph and basis (m = 200), C = 3, 50 seeds per label: Gaussian-fit priors
    from the seeds and the gamma > 0 solve with the choice of m from the priors (eps 0.1, r = 4)."""
    w = rwsynth.CFG2
    J, rid = rwsynth.phantom(w, 0)
    node, lab = rwsynth.seeds(w, rid, 0)
    Jd = torch.as_tensor(J, device=dev)
    g = rw.Graph(Jd, w.dims, w.conn, w.beta, dtype=torch.float32)
    t_pre, (Q, lam, einfo) = _sync_time(torch, lambda: rw.precompute_eig(g, w.m, tol=1e-5, max_iter=400), 1)
    gamma, eps, r = 1e-3, 0.1, 4
    ws = rw.SolveWorkspace()
    U = torch.empty((w.C, w.N), dtype=torch.float32, device=dev)

    def step():
        P = rw.priors_from_seeds(g, node, lab, w.C, dtype=torch.float32)
        return P, rw.solve_seeds_prior(g, Q, lam, node, lab, w.C, gamma, P, eps=eps, r=r, U=U, workspace=ws)[1]

    for _ in range(args.warmup):
        step()
    t, (P, info) = _sync_time(torch, step, args.steps)
    log(f"prior512: {t * 1e3:.2f} ms per priors + solve, m_used {info['m_used']}, g_worst/g_max "
        f"{info['g_worst']:.3e}/{info['g_max']:.3e}")
    parity = None
    cpu = None
    if not args.no_cpu:
        from oracle.fast_rw import fast_rw_prior
        from oracle.graph import Graph as OGraph
        from oracle.priors import choose_m_prior, gaussian_priors
        og = OGraph(J, w.dims, w.conn, w.beta)
        Qn, ln = Q.double().cpu().numpy().T, lam.cpu().numpy()
        t0 = time.perf_counter()
        Po = gaussian_priors(J, node, lab, w.C)
        m_o, _, _ = choose_m_prior(og, Qn, Po, eps=eps, r=r) if info["m_used"] < 20 else (None, None, None)
        Uo = fast_rw_prior(og, Qn, ln, node, lab, w.C, gamma, Po, m=info["m_used"])
        t_o = time.perf_counter() - t0
        parity = {"priors_vs_oracle_maxabs": float(np.abs(P.double().cpu().numpy().T - Po).max()),
                  "solve_vs_oracle_same_basis_maxabs": float(np.abs(U.double().cpu().numpy().T - Uo).max()),
                  "m_oracle": m_o}
        cpu = {"value": round(1.0 / t_o, 4), "unit": "solves/s", "cores": int(_cores()), "kind": "oracle",
               "sample": "one priors + gamma > 0 solve of this workload at the GPU's m (dense FP64 numpy)"}
    return _line("priors + gamma > 0 RW solves/s (choice of m from the priors)", round(1.0 / t, 2), "solves/s", args,
                 t * 1e3, "f32 graph/basis + f64 seed system, projection and prior fit",
                 {"workload": "2D 512x512 8-connected phantom, beta 90, FP32 basis m=200, C=3, 50 seeds/label, "
                              "Gaussian priors, gamma 1e-3, eps 0.1, r 4", "N": w.N, "m": w.m, "C": w.C,
                  "S": int(node.size)},
                 m_used=info["m_used"], g_max=info["g_max"], g_worst=info["g_worst"], precompute_s=round(t_pre, 2),
                 parity=parity, cpu_baseline=cpu)


def run_bank512(args, rw, rwsynth, torch, dev):
    """512 x 512, 8-connected, FP32, m = 200: bases precomputed for beta' in {45, 90, 180}; for beta = 150 the
    bank selection (diagonal update of each basis, eq. (27); the smallest quotient sum) and a solve with the
    chosen basis, against a solve with the basis computed for beta = 150 itself."""
    w = rwsynth.CFG2
    J, rid = rwsynth.phantom(w, 0)
    node, lab = rwsynth.seeds(w, rid, 0)
    Jd = torch.as_tensor(J, device=dev)
    betas, beta = (45.0, 90.0, 180.0), 150.0
    bank = []
    t0 = time.perf_counter()
    for b in betas:
        gb = rw.Graph(Jd, w.dims, w.conn, b, dtype=torch.float32)
        bank.append(rw.precompute_eig(gb, w.m, tol=1e-5, max_iter=400)[0].contiguous())
    torch.cuda.synchronize()
    t_bank = time.perf_counter() - t0
    g = rw.Graph(Jd, w.dims, w.conn, beta, dtype=torch.float32)
    ws = rw.SolveWorkspace()

    def step():
        idx, Q, lam, tr = rw.bank_select(g, bank)
        U, info = rw.solve_seeds(g, Q, lam, node, lab, w.C, eps=0.1, workspace=ws)
        return idx, tr, U, info

    for _ in range(args.warmup):
        step()
    t, (idx, tr, U, info) = _sync_time(torch, step, args.steps)
    t_sel, _ = _sync_time(torch, lambda: rw.bank_select(g, bank), args.steps)
    Qx, lamx, _ = rw.precompute_eig(g, w.m, tol=1e-5, max_iter=400)
    Ux, infox = rw.solve_seeds(g, Qx, lamx, node, lab, w.C, eps=0.1, workspace=ws)
    agree = float((U.argmax(dim=0) == Ux.argmax(dim=0)).double().mean())
    maxabs = float((U.double() - Ux.double()).abs().max())
    log(f"bank512: chose beta' = {betas[idx]} (sums {[round(x, 4) for x in tr]}), selection {t_sel * 1e3:.2f} ms, "
        f"selection + solve {t * 1e3:.2f} ms; labels agree with the beta = 150 basis on {agree:.4f} of the voxels")
    return _line("bank selection + RW solves/s (beta changed online, bases precomputed for three other beta)",
                 round(1.0 / t, 2), "solves/s", args, t * 1e3, "f32 graph/basis + f64 quotients and seed system",
                 {"workload": "2D 512x512 8-connected phantom, FP32 bases m=200 for beta' 45/90/180, beta 150, "
                              "C=3, 50 seeds/label, eps 0.1", "N": w.N, "m": w.m, "C": w.C, "S": int(node.size)},
                 chosen_beta=betas[idx], quotient_sums=tr, selection_ms=round(t_sel * 1e3, 3),
                 bank_precompute_s=round(t_bank, 2), m_used=info["m_used"],
                 vs_exact_beta_basis={"label_agreement": agree, "maxabs": maxabs, "m_used": infox["m_used"]})


def run_agg512(args, rw, rwsynth, torch, dev):
    """512 x 512, 8-connected, FP32 graph and basis (m = 200), C = 3, 50 seeds per label, aggregated into 2 x 2
    blocks (N_bar = N / 4): the aggregated graph, the eq. (33) transfer of the basis with Gram-Schmidt and the
    normalized-cut values, the seeds moved to their blocks, the solve on the blocks and the propagation back."""
    w = rwsynth.CFG2
    s = 2
    J, rid = rwsynth.phantom(w, 0)
    node, lab = rwsynth.seeds(w, rid, 0)
    Jd = torch.as_tensor(J, device=dev)
    g = rw.Graph(Jd, w.dims, w.conn, w.beta, dtype=torch.float32)
    t_pre, (Q, lam, _) = _sync_time(torch, lambda: rw.precompute_eig(g, w.m, tol=1e-5, max_iter=400), 1)
    Q = Q.contiguous()
    ws = rw.SolveWorkspace()

    def step():
        c = rw.aggregate(g, s)
        Qc, lamc = rw.aggregate_basis(g, c, s, Q)
        cn, cl = rw.aggregate_seeds(g, s, node, lab)
        Uc, info = rw.solve_seeds(c, Qc, lamc, cn, cl, w.C, eps=0.1, workspace=ws)
        return c, Qc, lamc, Uc, rw.prolong(g, s, Uc), info

    for _ in range(args.warmup):
        step()
    t, (c, Qc, lamc, Uc, U, info) = _sync_time(torch, step, args.steps)
    t_tr, _ = _sync_time(torch, lambda: rw.aggregate_basis(g, c, s, Q), args.steps)
    # the paper's baseline: a basis computed on the aggregated graph itself (not known before the aggregation)
    Qd, lamd, _ = rw.precompute_eig(c, w.m, tol=1e-5, max_iter=400)
    cn, cl = rw.aggregate_seeds(g, s, node, lab)
    Ud, infod = rw.solve_seeds(c, Qd, lamd, cn, cl, w.C, eps=0.1, workspace=ws)
    Uf, _ = rw.solve_seeds(g, Q, lam, node, lab, w.C, eps=0.1, workspace=ws)
    lab_t, lab_d, lab_f = Uc.argmax(dim=0), Ud.argmax(dim=0), Uf.argmax(dim=0)
    vs_direct = float((lab_t == lab_d).double().mean())
    vs_full = float((U.argmax(dim=0) == lab_f).double().mean())
    log(f"agg512: {t * 1e3:.2f} ms per aggregation + transfer + solve + propagation (transfer {t_tr * 1e3:.2f} ms), "
        f"N_bar {c.N}, m_used {info['m_used']}; labels agree with the direct basis on {vs_direct:.4f} of the blocks, "
        f"with the full-graph solve on {vs_full:.4f} of the voxels")
    parity = None
    cpu = None
    if not args.no_cpu:
        from oracle.aggregate import coarse_seeds, prolong, transfer_basis
        from oracle.fast_rw import fast_rw
        from oracle.graph import Graph as OGraph
        og = OGraph(J, w.dims, w.conn, w.beta)
        t0 = time.perf_counter()
        co, Qo, lamo = transfer_basis(og, Q.double().cpu().numpy().T, s)
        cno, clo = coarse_seeds(og, s, node, lab)
        Uo = prolong(og, s, fast_rw(co, Qo, lamo, cno, clo, w.C, m=info["m_used"]))
        t_o = time.perf_counter() - t0
        wv = c.view()["weight"].double().cpu().numpy()
        parity = {"weights_vs_oracle_maxrel": float(np.max(np.abs(wv[co.dir, co.tail] - co.w) / np.abs(co.w))),
                  "basis_vs_oracle_maxabs": float(np.abs(Qc.double().cpu().numpy().T - Qo).max()),
                  "lambda_vs_oracle_maxabs": float(np.abs(lamc.cpu().numpy() - lamo).max()),
                  "probabilities_vs_oracle_maxabs": float(np.abs(U.double().cpu().numpy().T - Uo).max())}
        cpu = {"value": round(1.0 / t_o, 4), "unit": "solves/s", "cores": int(_cores()), "kind": "oracle",
               "sample": "one aggregation + transfer + coarse solve + propagation of this workload (dense FP64 numpy)"}
    return _line("aggregated RW solves/s (eq. (33) transfer + solve on 2x2 blocks + propagation)", round(1.0 / t, 2),
                 "solves/s", args, t * 1e3, "f32 graph/basis + f64 Gram-Schmidt, quotients and seed system",
                 {"workload": "2D 512x512 8-connected phantom, beta 90, FP32 basis m=200, C=3, 50 seeds/label, "
                              "2x2 blocks", "N": w.N, "N_bar": c.N, "m": w.m, "C": w.C, "S": int(node.size)},
                 m_used=info["m_used"], transfer_ms=round(t_tr * 1e3, 3), precompute_s=round(t_pre, 2),
                 vs_direct_basis={"label_agreement": vs_direct, "m_used": infod["m_used"]},
                 vs_full_graph={"label_agreement": vs_full}, parity=parity, cpu_baseline=cpu)


def run_rwir96(args, rw, rwsynth, torch, dev):
    """96^3, 6-connected, beta 50, FP32 graph, BF16 basis (m = 200, precomputed in FP32), 21 x 21 x 9 = 3969
    displacement labels with BF16 priors, gamma 1, no seeds: the projection of the priors, the coefficients and
    the per-voxel labels fused with the reconstruction (U not formed)."""
    w = rwsynth.CFG6
    J, _ = rwsynth.phantom(w, 0)
    Jd = torch.as_tensor(J, device=dev)
    g = rw.Graph(Jd, w.dims, w.conn, w.beta, dtype=torch.float32)
    t_pre, (Q, lam, einfo) = _sync_time(torch, lambda: rw.precompute_eig(g, w.m, tol=1e-5, max_iter=400), 1)
    Qb = rw.convert_block(Q.contiguous(), torch.bfloat16)
    labels = rwsynth.displacement_labels(rwsynth.CFG6_EXTENT)
    field = rwsynth.displacement_field(w.dims, rwsynth.CFG6_EXTENT, rwsynth.CFG6_ID)
    P = rwsynth.displacement_priors_torch(torch.as_tensor(field, device=dev), torch.as_tensor(labels, device=dev),
                                          dtype=torch.bfloat16, chunk=2048)
    C, N, gamma = labels.shape[0], w.N, rwsynth.CFG6_GAMMA
    ws = rw.SolveWorkspace()

    def step():
        return rw.solve_priors(g, Qb, lam, P, gamma, want_U=False, want_labels=True, workspace=ws)

    for _ in range(args.warmup):
        step()
    t, (_, lab, prob, info) = _sync_time(torch, step, args.steps)
    _, (_, lab_e, _, info_e) = _sync_time(torch, lambda: rw.solve_priors(g, Qb, lam, P, gamma, eps=0.1, r=4,
                                                                         want_U=False, want_labels=True,
                                                                         workspace=ws), 1)
    p_bytes = N * C * 2
    KR = (w.m + 31) // 32 * 32
    KC = 16 * 13
    flops = 2.0 * N * C * (KC + KR)
    log(f"rwir96: {t * 1e3:.2f} ms per solve (N {N}, C {C}, m {info['m_used']}); priors read at "
        f"{p_bytes / t / 1e9:.0f} GB/s over the whole call; eps 0.1 chooses m = {info_e['m_used']}")
    parity = None
    cpu = None
    if not args.no_cpu:
        from oracle.graph import Graph as OGraph
        from oracle.rwir import rwir_coefficients
        og = OGraph(J, w.dims, w.conn, w.beta)
        Qn = Qb.double().cpu().numpy().T
        rng = np.random.default_rng(5)
        rows = np.sort(rng.choice(N, size=2048, replace=False))
        t0 = time.perf_counter()
        # the oracle's projection streamed over voxel chunks of the same BF16 priors (C x N on the device)
        from oracle.eigen import insert_null
        Qi, li = insert_null(Qn, lam.cpu().numpy(), og.ghat())
        hs = og.hat_scale()
        Z = np.zeros((w.m, C))
        for a in range(0, N, 32768):
            b = min(N, a + 32768)
            Pc = P[:, a:b].double().cpu().numpy().T
            Z += Qi[a:b].T @ (hs[a:b, None] * Pc)
        Y = (gamma / (li + gamma))[:, None] * Z
        t_z = time.perf_counter() - t0
        t1 = time.perf_counter()
        Ur = (Qi[rows] @ Y) / hs[rows, None]
        t_r = time.perf_counter() - t1
        top = Ur.max(axis=1)
        lg = lab.cpu().numpy()[rows]
        at = Ur[np.arange(rows.size), lg]
        parity = {"sampled_voxels": int(rows.size),
                  "label_value_gap_max": float((top - at).max()),
                  "prob_vs_oracle_maxabs": float(np.abs(prob.double().cpu().numpy()[rows] - at).max()),
                  "labels_equal_oracle_argmax": float(np.mean(np.argmax(Ur, axis=1) == lg))}
        t_o = t_z + t_r * N / rows.size
        cpu = {"value": round(1.0 / t_o, 5), "unit": "solves/s", "cores": int(_cores()), "kind": "oracle",
               "sample": f"the oracle's full projection of the priors ({t_z:.1f} s, FP64 numpy) plus its labels on "
                         f"{rows.size} voxels ({t_r:.2f} s), the latter scaled to all {N} voxels"}
    return _line("RW solves/s driven by priors alone at registration label counts (labels per voxel)",
                 round(1.0 / t, 2), "solves/s", args, t * 1e3,
                 "bf16 basis and priors on the matrix cores (f32 accumulation) + f64 coefficients",
                 {"workload": "3D 96^3 6-connected phantom, beta 50, BF16 basis m=200, 21x21x9 = 3969 displacement "
                              "labels (BF16 priors), gamma 1, no seeds", "N": N, "m": w.m, "C": C},
                 m_used=info["m_used"], m_chosen_eps_0_1=info_e["m_used"],
                 effective={"prior_bytes_per_solve": p_bytes, "prior_gbs_whole_call": round(p_bytes / t / 1e9, 1),
                            "mfma_flop_per_solve": flops,
                            "mfma_tflops_whole_call": round(flops / t / 1e12, 1)},
                 precompute_s=round(t_pre, 2), parity=parity, cpu_baseline=cpu)


MODES = {"small64": run_small64, "volume128": run_volume128, "batch64": run_batch64, "grad96": run_grad96,
         "prior512": run_prior512, "bank512": run_bank512,
         "agg512": run_agg512, "rwir96": run_rwir96}


if __name__ == "__main__":
    main()
