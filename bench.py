#!/usr/bin/env python3
"""Benchmark of the even-odd Wilson-clover solve on one MI355X.

One step = one complete solve of M x = b to a 1e-10 FP64 true residual on
the 32^3x64 lattice (kappa = 0.135, csw = 1.0, smooth SU(3) links with
eps = 0.3, Gaussian source), with b and x resident in HBM: mixed-precision
CG on the normal equations of the Schur operator (FP16 inner iteration with
per-site FP32 scales by default, FP32 inner vectors, FP64 reliable updates,
FP64 final residual).

Printed (one JSON line):
  autotune      the tile tuner's choice (lq_tune_tiles) for the single-RHS
                numbering and the 12-RHS numbering, every candidate's time and
                the spread; the benchmark's contexts use the chosen tiles;
  value         whole-solve throughput: algorithmic bytes of every kernel the
                solve launched / wall time of the timed steps, in GB/s;
  ms_per_step   wall time per solve;
  roofline      the solve's dominant kernel (largest share of kernel time),
                timed with HIP events inside the library during one
                profiled solve, priced against the 8 TB/s HBM peak;
  plain_fp64    the same solve with plain FP64 CG, for comparison;
  dslash_gbs    stand-alone hopping-term sweeps per precision over three
                rotated copies of the fields (HIP events per launch), beside the
                library's 16-byte streaming copy (hbm_copy), the achievable HBM
                bandwidth;
  fused_expressions
                the SU(3) array product of the paper's worked example and a
                three-factor product fused into one pass against two passes;
  batched_12rhs the 12 spin-colour point sources of a propagator solved
                together through the multi-RHS operator (FP16 on the matrix
                cores) as independent recurrences and as one block CG, beside
                one point source solved alone (plain FP64 and mixed FP16)
                scaled by 12;
  learned_preconditioner
                a 4-layer gauge-covariant net trained on the GPU on 2000
                (source, solution) pairs the solver generated on a 16^3x32
                field (weights kept by held-out solve iterations), then used on
                the benchmark's 32^3x64 field in flexible CG, FGMRES and
                FGMRES-DR, beside its Neumann start;
  uneven_batch  eight lattices of different volumes and kappas solved as one
                batch, beside the same solves one after another;
  sap_fgcr      the paper's own solver on the benchmark system: FGCR with the
                SAP preconditioner (FP32 block MR, FP64 restarts), the same
                preconditioner in FGMRES with deflated restarting, both again
                with the block solves' operator in FP16 staged in LDS, and with
                MR on the even-odd reduced block operator, and one SAP
                application alone in each form;
  cpu_baseline  the FP64 oracle timed on the host on a bounded sample.

roofline.traffic is the HBM traffic per launch of the roofline kernel from
the committed counter summary (profiles/traffic_*.txt), reported only while
the library sources still match the digest recorded there.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

KAPPA, CSW, TOL = 0.135, 1.0, 1e-10
KNAMES = ["hop_oe+clover_inv", "hop_eo+clover+norm", "hop_oe_dag+clover_inv",
          "hop_eo_dag+clover+cg_update", "p_update"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def batched_point_sources(lq, lat, torch, dims):
    """The 12 point sources at the origin solved as one batch, against one of
    them solved alone (plain FP64 CG and mixed FP16 CG) times 12."""
    from gen import fields
    b = fields.point_sources_12(dims)
    db = lat.to_device(b, lq.FULL, lq.F64)
    dx = lat.new_field(lq.FULL, lq.F64, 12)
    lat.solve_device(dx, db, KAPPA, CSW, TOL, nrhs=12, inner_prec=lq.F16, batched=1)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = lat.solve_device(dx, db, KAPPA, CSW, TOL, nrhs=12, inner_prec=lq.F16, batched=1)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    one = lat.field_bytes(lq.FULL, lq.F64)
    db1, dx1 = db[:one], lat.new_field(lq.FULL, lq.F64)
    single = {}
    for name, prec in (("plain_fp64", lq.F64), ("mixed_f16", lq.F16)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = lat.solve_device(dx1, db1, KAPPA, CSW, TOL, inner_prec=prec)[0]
        torch.cuda.synchronize()
        single[name] = {"ms": round((time.perf_counter() - t0) * 1e3, 2),
                        "iterations": r.iterations, "true_residual": r.true_residual}
    lat.solve_device(dx, db, KAPPA, CSW, TOL, nrhs=12, inner_prec=lq.F16, batched=2)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rblk = lat.solve_device(dx, db, KAPPA, CSW, TOL, nrhs=12, inner_prec=lq.F16, batched=2)
    torch.cuda.synchronize()
    tblk = time.perf_counter() - t0
    out = {"rhs": 12, "sources": "point sources at the origin, one per (spin, colour)",
           "block_cg": {"solve_ms": round(tblk * 1e3, 2), "iterations": rblk[0].iterations,
                        "reliable_updates": rblk[0].reliable_updates,
                        "fallback": rblk[0].fallback,
                        "max_true_residual": max(r.true_residual for r in rblk),
                        "operator_applications_vs_batched": None},
           "solve_ms": round(tb * 1e3, 2), "ms_per_rhs": round(tb * 1e3 / 12, 2),
           "iterations": reps[0].iterations, "reliable_updates": reps[0].reliable_updates,
           "fallback": reps[0].fallback,
           "max_true_residual": max(r.true_residual for r in reps),
           "one_source_alone": single,
           "speedup_vs_12x_plain_fp64": round(12 * single["plain_fp64"]["ms"] / (tb * 1e3), 3),
           "speedup_vs_12x_mixed_f16": round(12 * single["mixed_f16"]["ms"] / (tb * 1e3), 3)}
    out["block_cg"]["operator_applications_vs_batched"] = round(
        rblk[0].iterations / max(1, reps[0].iterations), 3)
    out["block_cg"]["speedup_vs_12x_mixed_f16"] = round(
        12 * single["mixed_f16"]["ms"] / (tblk * 1e3), 3)
    del db, dx, dx1
    return out


def uneven_batch(lq, torch):
    """Eight independent solves on lattices from 8^4 to 24^3x48 (kappa in
    [0.130, 0.136], csw = 1, smooth links, Gaussian sources) as one uneven
    batch, against the same eight solved one after another."""
    from gen import fields
    spec = fields.uneven_batch()
    t0 = time.perf_counter()
    lats, db, dx = [], [], []
    for dims, kappa, gs, ss in spec:
        lat = lq.Lattice(dims)
        lat.upload_gauge(fields.gauge_field(dims, "smooth", gs))
        lat.set_clover(kappa, CSW)
        lats.append(lat)
        db.append(lat.to_device(fields.gaussian_spinor(dims, ss), lq.FULL, lq.F64))
        dx.append(lat.new_field(lq.FULL, lq.F64))
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    kap = [k for _, k, _, _ in spec]
    csw = [CSW] * len(spec)
    ens = lq.Ensemble(lats)
    out = {"members": ["x".join(map(str, d)) for d, *_ in spec],
           "kappa": [round(k, 5) for k in kap], "even_sites": sum(l.volume // 2 for l in lats),
           "inputs_s": round(t_gen, 1)}
    for name, prec in (("batch_mixed_f16", lq.F16), ("batch_plain_f64", lq.F64)):
        tune = ens.tune(prec)
        ens.solve_device(dx, db, kap, csw, TOL, inner_prec=prec)  # warm-up: graphs, clover
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps, er = ens.solve_device(dx, db, kap, csw, TOL, inner_prec=prec)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        out[name] = {"ms": round(ms, 2), "tile_sites": tune["tile_sites"],
                     "tune_ms_per_iteration": [round(t, 4) for t in tune["tune_ms"]],
                     "graph_captures": er["graph_captures"], "replays": er["replays"],
                     "iterations": [r.iterations for r in reps],
                     "reliable_updates": [r.reliable_updates for r in reps],
                     "fallbacks": sum(r.fallback for r in reps),
                     "max_true_residual": max(r.true_residual for r in reps),
                     "GB/s": round(er["bytes"] / (ms * 1e-3) / 1e9, 1)}
    for name, prec in (("sequential_plain_f64", lq.F64), ("sequential_mixed_f16", lq.F16)):
        for j, lat in enumerate(lats):  # warm-up: work fields and graphs of every lattice
            lat.solve_device(dx[j], db[j], kap[j], CSW, TOL, inner_prec=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = [lat.solve_device(dx[j], db[j], kap[j], CSW, TOL, inner_prec=prec)[0]
                for j, lat in enumerate(lats)]
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        out[name] = {"ms": round(ms, 2), "iterations": [r.iterations for r in reps],
                     "max_true_residual": max(r.true_residual for r in reps)}
    b16 = out["batch_mixed_f16"]["ms"]
    out["speedup_vs_sequential_plain_f64"] = round(out["sequential_plain_f64"]["ms"] / b16, 3)
    out["speedup_vs_sequential_mixed_f16"] = round(out["sequential_mixed_f16"]["ms"] / b16, 3)
    out["batch_plain_vs_sequential_plain"] = round(
        out["sequential_plain_f64"]["ms"] / out["batch_plain_f64"]["ms"], 3)
    ens.close()
    del db, dx
    return out


def learned_preconditioner(lq, lat, torch, db_bench, npairs, epochs):
    """Train the net on (source, FP64 solution) pairs the solver generates on a
    16^3x32 field (its own gauge field and sources), one epoch at a time.
    After every epoch, flexible CG with the current weights solves a
    held-out source on the training lattice; the weights with the fewest
    iterations are kept, the Neumann start among the candidates, so the net
    carried to the benchmark is never worse than its start on held-out data.
    Then the benchmark system (its source on the device, db_bench) is solved
    with the kept net, with its Neumann start, and with FGMRES-DR."""
    import numpy as np
    from gen import fields
    dt = (16, 16, 16, 32)
    t0 = time.perf_counter()
    ut = fields.gauge_field(dt, "smooth", fields.SEED_TRAIN_FIELD)
    tl = lq.Lattice(dt)
    tl.upload_gauge(ut)
    tl.set_clover(KAPPA, CSW)
    vh = tl.volume // 2
    rng = np.random.default_rng(fields.SEED_TRAIN_SOURCE)
    fb32 = tl.field_bytes(lq.EVEN, lq.F32)
    h64 = tl.field_bytes(lq.EVEN, lq.F64)
    db, dx = tl.new_field(lq.EVEN, lq.F32, npairs), tl.new_field(lq.EVEN, lq.F32, npairs)
    dB, dX = tl.new_field(lq.FULL, lq.F64), tl.new_field(lq.FULL, lq.F64)  # odd half of dB: 0
    for i in range(npairs):
        be = (rng.standard_normal((vh, 4, 3)) + 1j * rng.standard_normal((vh, 4, 3))) / np.sqrt(2)
        tl.to_device(be, lq.EVEN, lq.F64, out=dB[:h64])  # b = (b_e, 0): x_e = Mhat^-1 b_e
        tl.solve_device(dX, dB, KAPPA, CSW, TOL, inner_prec=lq.F16)
        xe = tl.to_host(dX[:h64], lq.EVEN, lq.F64)
        tl.to_device(be, lq.EVEN, lq.F32, out=db[i * fb32:(i + 1) * fb32])
        tl.to_device(xe, lq.EVEN, lq.F32, out=dx[i * fb32:(i + 1) * fb32])
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    ntr = max(1, int(0.9 * npairs))
    nv = npairs - ntr
    net = lq.Net(tl, 4)
    net.init_neumann(KAPPA)
    w0 = net.get_weights()
    l0, _ = net.loss_grad(db, dx, ntr)
    v0 = net.loss_grad(db[ntr * fb32:], dx[ntr * fb32:], nv)[0] if nv else None
    b_sel = fields.gaussian_spinor(dt, fields.SEED_TRAIN_SOURCE + 99999)  # held-out source

    def sel_iterations(wts):  # resets the Adam state: callers restore it
        net.set_weights(wts)
        _, rep = net.solve(b_sel, KAPPA, CSW, TOL, solver=lq.FCG_NET)
        return rep[0].iterations + (10 ** 6 if rep[0].fallback else 0)

    best_w, best_it, best_at = w0, sel_iterations(w0), "start"
    sel = [best_it]
    net.set_weights(w0)
    hist = []
    t_train = 0.0
    # each epoch runs over the training pairs in `chunks` consecutive slices
    # (one shuffled pass per slice), and the selection looks after each
    chunks = 8
    bounds = [ntr * c // chunks for c in range(chunks + 1)]
    ck = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"lq_net_{os.getpid()}.ckpt")
    for e in range(epochs):
        ep_loss = []
        for c in range(chunks):
            lo, hi = bounds[c], bounds[c + 1]
            if hi <= lo:
                continue
            t1 = time.perf_counter()
            ep_loss += [float(h) * (hi - lo) for h in
                        net.train(db[lo * fb32:], dx[lo * fb32:], hi - lo, epochs=1, batch=8,
                                  lr=1e-3, seed=1 if e == 0 and c == 0 else 0)]
            torch.cuda.synchronize()
            t_train += time.perf_counter() - t1
            w_e = net.get_weights()
            # checkpoint the training state: selection solves leave the Adam state alone
            net.save(ck)
            it = sel_iterations(w_e)
            net.load(ck)
            sel.append(it)
            if it < best_it:
                best_w, best_it, best_at = w_e, it, f"epoch {e + 1}, slice {c + 1}"
        hist.append(sum(ep_loss) / ntr)
    if os.path.exists(ck):
        os.remove(ck)
    l1, _ = net.loss_grad(db, dx, ntr)
    v1 = net.loss_grad(db[ntr * fb32:], dx[ntr * fb32:], nv)[0] if nv else None
    del db, dx, dB, dX, net, tl
    bn = lq.Net(lat, 4)
    out = {"layers": 4, "train_lattice": list(dt), "pairs": npairs, "train_pairs": ntr,
           "epochs": epochs, "pair_generation_s": round(t_pairs, 2), "training_s": round(t_train, 2),
           "loss_train": [round(l0, 5), round(l1, 5)],
           "loss_valid": [round(v0, 5), round(v1, 5)] if nv else None,
           "loss_history": [round(float(h), 5) for h in hist],
           "selection": {"held_out_fcg_iterations": sel, "kept": best_at,
                         "rule": f"fewest flexible-CG iterations on a held-out 16^3x32 source, "
                                 f"checked at the start (the Neumann series) and after each "
                                 f"1/{chunks} of every epoch"},
           "solves": {}}
    b_host = lat.to_host(db_bench, lq.FULL, lq.F64)
    for name, wts, kind, kw in (("fcg_trained", best_w, lq.FCG_NET, {}),
                                ("fcg_initial", w0, lq.FCG_NET, {}),
                                ("fgmres_trained", best_w, lq.FGMRES_NET, {}),
                                ("fgmres_dr_trained", best_w, lq.FGMRES_NET,
                                 {"restart": 70, "deflate": 10})):
        bn.set_weights(wts)
        t1 = time.perf_counter()
        _, rep = bn.solve(b_host, KAPPA, CSW, TOL, solver=kind, **kw)
        dt_s = time.perf_counter() - t1
        out["solves"][name] = {"ms": round(dt_s * 1e3, 1), "iterations": rep[0].iterations,
                               "restarts": rep[0].reliable_updates, "fallback": rep[0].fallback,
                               "dslash_equivalents": rep[0].dslash_calls,
                               "true_residual": rep[0].true_residual}
    # the net application alone, in the solvers' FP16 form, on the even half of b
    dn = lat.to_device(lat.to_host(db_bench[:lat.field_bytes(lq.EVEN, lq.F64)], lq.EVEN, lq.F64),
                       lq.EVEN, lq.F32)
    dy = lat.new_field(lq.EVEN, lq.F32)
    bn.set_weights(best_w)
    for _ in range(3):
        bn.apply(dy, dn, fp16=True)
    a = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(10):
        bn.apply(dy, dn, fp16=True)
    e.record()
    torch.cuda.synchronize()
    out["net_apply_fp16_ms"] = round(a.elapsed_time(e) / 10, 3)
    del dn, dy, bn
    return out


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when the sources changed since it was taken."""
    from paper_1103_1363_amd.prof_summary import source_digest
    import glob
    digest = source_digest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.txt"))):
        lines = open(path).read().splitlines()
        rec = [ln.split(":", 1)[1].strip() for ln in lines if ln.startswith("# source_digest:")]
        if not rec or rec[0] != digest:
            continue
        for ln in lines:
            parts = ln.rsplit(None, 3)
            if len(parts) == 4 and parts[0].replace(" ", "") == kernel.replace(" ", ""):
                return {"bytes_per_launch": float(parts[2]) + float(parts[3]),
                        "fetch_bytes": float(parts[2]), "write_bytes": float(parts[3]),
                        "source": os.path.basename(path)}
    return None


def sap_fgcr(lq, lat, torch, db, block, ncycles, nmr, restart, dr_m=70, dr_k=10):
    """The paper's own solver on the benchmark system: FGCR with the SAP
    preconditioner (FP32 block MR and inner FGCR, FP64 restarts), after one
    warm-up solve; the same preconditioner in FGMRES with deflated
    restarting (Krylov dimension dr_m including dr_k deflated vectors, the
    paper's 70 and 10); and one SAP application alone, with the algorithmic
    bytes of its kernels (the library's own count)."""
    dx = lat.new_field(lq.FULL, lq.F64)
    lat.solve_sap_device(dx, db, KAPPA, CSW, TOL, block, ncycles, nmr, restart)
    out = {"block": list(block), "ncycles": ncycles, "nmr": nmr}
    for name, kw in (("fgcr", {"restart": restart}),
                     ("fgmres_dr", {"restart": dr_m, "deflate": dr_k}),
                     ("fgcr_fp16_blocks", {"restart": restart, "block_fp16": True}),
                     ("fgmres_dr_fp16_blocks", {"restart": dr_m, "deflate": dr_k,
                                                "block_fp16": True}),
                     ("fgcr_fp16_eo_blocks", {"restart": restart, "block_fp16": True,
                                              "block_eo": True}),
                     ("fgmres_dr_fp16_eo_blocks", {"restart": dr_m, "deflate": dr_k,
                                                   "block_fp16": True, "block_eo": True}),
                     ("fgcr_fp16_eo_blocks_4mr_restart24",
                      {"restart": 24, "block_fp16": True, "block_eo": True, "nmr": 4})):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kw_nmr = kw.pop("nmr", nmr)
        rep = lat.solve_sap_device(dx, db, KAPPA, CSW, TOL, block, ncycles, kw_nmr, **kw)
        if kw_nmr != nmr:
            kw["nmr"] = kw_nmr
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        out[name] = {**kw, "ms": round(ms, 1), "steps": rep.iterations,
                     "restarts": rep.reliable_updates, "true_residual": rep.true_residual,
                     "GB/s": round(rep.bytes / (rep.seconds if rep.seconds > 0 else ms / 1e3)
                                   / 1e9, 1)}
    e = lat.new_field(lq.FULL, lq.F32)
    y = lat.new_field(lq.FULL, lq.F32)
    e.copy_(lat.to_device(lat.to_host(db, lq.FULL, lq.F64), lq.FULL, lq.F32))
    for name, fp16, eo in (("sap_apply_ms", False, False),
                           ("sap_apply_fp16_blocks_ms", True, False),
                           ("sap_apply_fp16_eo_blocks_ms", True, True)):
        lat.sap_apply(y, e, block, ncycles, nmr, block_fp16=fp16, block_eo=eo)
        a = torch.cuda.Event(enable_timing=True)
        z = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(5):
            lat.sap_apply(y, e, block, ncycles, nmr, block_fp16=fp16, block_eo=eo)
        z.record()
        torch.cuda.synchronize()
        out[name] = round(a.elapsed_time(z) / 5, 3)
    return out


def cpu_info():
    model, cores = "unknown", os.cpu_count() or 1
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    return model, cores


def cpu_baseline(u, b, dims, gpu_iters):
    """The FP64 oracle (NumPy) on the host, timed on bounded samples of the
    workloads (NumPy runs them on one thread: its element-wise and einsum
    kernels do not spread over cores):
      * one even-odd hopping sweep H_eo of the 32^3x64 benchmark field, priced
        with the same 1152 algorithmic bytes per output site as the GPU sweep
        (the value), and one of a 16^3x32 field;
      * the whole 4^4 Wilson solve of the small configuration (even-odd CGNR
        to 1e-10);
      * one CGNR iteration on the 16^3x32 Schur operator (one application of
        Mhat and one of Mhat^+; the vector updates are negligible beside
        them), from which whole solves are extrapolated with the iteration
        counts the GPU solves of this run needed (gpu_iters: name -> (sites
        factor relative to 16^3x32, iterations)); each extrapolation says so."""
    import numpy as np
    from oracle import dirac, evenodd
    from oracle import solvers
    from gen import fields
    model, ncpu = cpu_info()
    e, o = evenodd.split(b, dims)
    t0 = time.perf_counter()
    y = dirac.hop(u, evenodd.join(None, o, dims))
    evenodd.split(y, dims)
    dt = time.perf_counter() - t0
    vh = e.shape[0]
    d16 = (16, 16, 16, 32)
    vh16 = 16 * 16 * 16 * 32 // 2
    u16 = fields.gauge_field(d16, "smooth", fields.SEED_GAUGE + 1)
    b16 = fields.gaussian_spinor(d16, fields.SEED_SOURCE + 1)
    t0 = time.perf_counter()
    dirac.hop(u16, evenodd.join(None, evenodd.split(b16, d16)[1], d16))
    dt16 = time.perf_counter() - t0
    wc16 = evenodd.WilsonClover(u16, KAPPA, CSW)
    bh16 = wc16.prepare_source(b16)
    t0 = time.perf_counter()
    z = wc16.schur(wc16.schur(bh16), dagger=True)
    dit = time.perf_counter() - t0
    del z
    d4 = (4, 4, 4, 4)
    u4 = fields.gauge_field(d4, "haar", fields.SEED_GAUGE)
    b4 = fields.gaussian_spinor(d4, fields.SEED_SOURCE)
    wc = evenodd.WilsonClover(u4, 0.12, 0.0)
    t0 = time.perf_counter()
    x4, info = solvers.solve_evenodd(wc, b4, tol=1e-10)
    dt4 = time.perf_counter() - t0
    extrap = {name: {"seconds": round(dit * f * it, 1), "iterations": it,
                     "from": f"{f:g} x the 16^3x32 CGNR iteration x {it} iterations "
                             "(the GPU plain FP64 solve's count)"}
              for name, (f, it) in gpu_iters.items()}
    return {"value": round(1152 * vh / dt / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "cpu_model": model, "host_cpus": ncpu, "seconds": round(dt, 2),
            "sample": "one FP64 even-odd hopping-term sweep (H_eo, 1152 algorithmic bytes per "
                      "output site) of the 32^3x64 field by the NumPy oracle, single thread",
            "dslash_16x16x16x32": {"seconds": round(dt16, 3),
                                   "GB/s": round(1152 * vh16 / dt16 / 1e9, 3)},
            "cgnr_iteration_16x16x16x32": {"seconds": round(dit, 2),
                                           "what": "Mhat then Mhat^+ on the 16^3x32 clover "
                                                   "Schur operator"},
            "solve_4x4x4x4_wilson": {"seconds": round(dt4, 3), "iterations": info.iterations,
                                     "true_residual": info.true_residual},
            "extrapolated_solves": extrap}


def config_16(lq, torch):
    """The 16^3x32 configuration (kappa 0.135, csw 1, smooth links, Gaussian
    source): FP32 inner iteration with FP64 reliable updates against plain
    FP64 CG, and BiCGStab on the Schur operator (FP32 inner and FP64).  Its
    fields (about 0.1 GB) stay in the 256 MB last-level cache, so its rates
    are cache-resident, not HBM rates."""
    from gen import fields
    d16 = (16, 16, 16, 32)
    u16 = fields.gauge_field(d16, "smooth", fields.SEED_GAUGE + 1)
    b16 = fields.gaussian_spinor(d16, fields.SEED_SOURCE + 1)
    lat = lq.Lattice(d16)
    lat.upload_gauge(u16)
    lat.set_clover(KAPPA, CSW)
    db = lat.to_device(b16, lq.FULL, lq.F64)
    dx = lat.new_field(lq.FULL, lq.F64)
    out = {"lattice": list(d16), "note": "working set resident in the last-level cache"}
    for name, prec in (("mixed_f32", lq.F32), ("mixed_f16", lq.F16), ("plain_fp64", lq.F64)):
        lat.solve_device(dx, db, KAPPA, CSW, TOL, inner_prec=prec)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = lat.solve_device(dx, db, KAPPA, CSW, TOL, inner_prec=prec)[0]
        torch.cuda.synchronize()
        out[name] = {"ms": round((time.perf_counter() - t0) * 1e3, 2), "iterations": r.iterations,
                     "reliable_updates": r.reliable_updates, "fallback": r.fallback,
                     "true_residual": r.true_residual}
    out["speedup_f32_vs_plain_fp64"] = round(out["plain_fp64"]["ms"] / out["mixed_f32"]["ms"], 3)
    for name, prec in (("bicgstab_f32", lq.F32), ("bicgstab_f64", lq.F64)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = lat.solve_device(dx, db, KAPPA, CSW, TOL, solver=lq.BICGSTAB, inner_prec=prec)[0]
        torch.cuda.synchronize()
        out[name] = {"ms": round((time.perf_counter() - t0) * 1e3, 2), "iterations": r.iterations,
                     "reliable_updates": r.reliable_updates, "fallback": r.fallback,
                     "true_residual": r.true_residual}
    del lat, db, dx
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--inner", choices=["f32", "f16"], default="f16")
    ap.add_argument("--dims", default="32,32,32,64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-net", action="store_true")
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--no-sap", action="store_true")
    ap.add_argument("--net-pairs", type=int, default=2000)
    ap.add_argument("--net-epochs", type=int, default=8)
    ap.add_argument("--gauge-cache", default=None,
                    help="an .npy file holding the benchmark gauge field (written if absent)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}): the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if world != 1:
        print("bench.py is single-process; run it without torch.distributed", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from gen import fields
    from paper_1103_1363_amd import lq

    dims = tuple(int(x) for x in a.dims.split(","))
    inner = {"f32": lq.F32, "f16": lq.F16}[a.inner]
    log(f"generating the {dims} smooth gauge field and source")
    if a.gauge_cache and os.path.exists(a.gauge_cache):
        u = np.load(a.gauge_cache)
    else:
        u = fields.gauge_field(dims, "smooth", fields.SEED_GAUGE + 2)
        if a.gauge_cache:
            np.save(a.gauge_cache, u)
    b = fields.gaussian_spinor(dims, fields.SEED_SOURCE + 2)

    log("tile tuner: the inner-precision Schur operator and the 12-RHS operator")
    t_tune = time.perf_counter()
    tune_one = lq.tune_tiles(dims, inner, 1)
    tune_12 = lq.tune_tiles(dims, lq.F16X, 12)
    t_tune = time.perf_counter() - t_tune
    tiling = {"tile_sites": int(tune_one.target[tune_one.best]),
              "mr_tile_sites": int(tune_12.target[tune_12.best])}
    lat = lq.Lattice(dims, **tiling)
    lat.upload_gauge(u)
    lat.set_clover(KAPPA, CSW)
    db = lat.to_device(b, lq.FULL, lq.F64)
    dx = lat.new_field(lq.FULL, lq.F64)
    torch.cuda.synchronize()

    log(f"warmup: {a.warmup} solve(s), inner {a.inner}")
    for _ in range(a.warmup):
        lat.solve_device(dx, db, KAPPA, CSW, TOL, inner_prec=inner)
    torch.cuda.synchronize()
    log(f"timed: {a.steps} solve(s)")
    t0 = time.perf_counter()
    reps = []
    for _ in range(a.steps):
        reps += lat.solve_device(dx, db, KAPPA, CSW, TOL, inner_prec=inner)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    total_bytes = sum(r.bytes for r in reps)
    value = total_bytes / wall / 1e9
    r0 = reps[-1]
    log(f"solve: {wall / a.steps * 1e3:.1f} ms, {r0.iterations} iterations, "
        f"{r0.reliable_updates} reliable updates, residual {r0.true_residual:.2e}")

    result = {
        "metric": "Dslash GB/s & %HBM peak; solve time to 1e-10 residual, plain vs mixed/learned",
        "value": round(value, 1),
        "value_is": "whole-solve algorithmic GB/s of the mixed FP16/FP64 solve (all its kernels' "
                    "compulsory bytes / wall time); the stand-alone Dslash rates and their "
                    "fractions of the 8 TB/s HBM peak are under dslash_gbs / dslash_frac_hbm",
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(wall / a.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": a.inner,
        "data": "synthetic",
        "config": {
            "workload": f"{'x'.join(map(str, dims))} even-odd Wilson-clover solve to 1e-10 "
                        f"(kappa={KAPPA}, csw={CSW}, smooth SU(3) links eps=0.3, Gaussian "
                        f"source), CG on the Schur normal equations, {a.inner} inner "
                        "iteration with FP64 reliable updates",
            "lattice": list(dims), "kappa": KAPPA, "csw": CSW, "tol": TOL,
            "rhs": 1, "parallelism": "single GPU",
        },
        "solve": {"iterations": r0.iterations, "reliable_updates": r0.reliable_updates,
                  "fallback": r0.fallback, "true_residual": r0.true_residual,
                  "seconds_inside_library": round(r0.seconds, 4),
                  "algorithmic_GB": round(r0.bytes / 1e9, 2)},
    }

    def spread(rep):
        us = [rep.us[i] for i in range(rep.ncand)]
        return round(max(us) / min(us), 3)

    result["autotune"] = {
        "what": "largest tile (sites of one parity) of the single-RHS numbering, timed on the "
                f"{a.inner} Schur operator, and of the 12-RHS numbering, timed on the 12-RHS "
                "Schur operator; unit links on scratch contexts, 20 applications each",
        "single_rhs": {**tune_one.as_dict(), "spread_slowest_over_fastest": spread(tune_one)},
        "rhs12": {**tune_12.as_dict(), "spread_slowest_over_fastest": spread(tune_12)},
        "seconds": round(t_tune, 2)}

    x_mixed = lat.to_host(dx, lq.FULL, lq.F64)
    if not a.no_plain:
        log("plain FP64 solve for comparison")
        dx2 = lat.new_field(lq.FULL, lq.F64)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        rp = lat.solve_device(dx2, db, KAPPA, CSW, TOL, inner_prec=lq.F64)[0]
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp
        x_plain = lat.to_host(dx2, lq.FULL, lq.F64)
        err = float(np.linalg.norm(x_mixed - x_plain) / np.linalg.norm(x_plain))
        result["plain_fp64"] = {"ms": round(tp * 1e3, 2), "iterations": rp.iterations,
                                "true_residual": rp.true_residual,
                                "GB/s": round(rp.bytes / tp / 1e9, 1)}
        result["speedup_vs_plain_fp64"] = round(tp / (wall / a.steps), 3)
        result["mixed_vs_plain_rel_error"] = err
        log("BiCGStab on the Schur operator, same inner precision and plain FP64")
        bi = {}
        for name, prec in ((a.inner, inner), ("f64", lq.F64)):
            # no warm-up: on this indefinite system BiCGStab runs for seconds
            torch.cuda.synchronize()
            tb = time.perf_counter()
            rb = lat.solve_device(dx2, db, KAPPA, CSW, TOL, solver=lq.BICGSTAB,
                                  inner_prec=prec)[0]
            torch.cuda.synchronize()
            tb = time.perf_counter() - tb
            bi[name] = {"ms": round(tb * 1e3, 2), "iterations": rb.iterations,
                        "reliable_updates": rb.reliable_updates, "fallback": rb.fallback,
                        "true_residual": rb.true_residual, "GB/s": round(rb.bytes / tb / 1e9, 1)}
        result["bicgstab"] = bi
        del dx2

    log("profiled solve (per-kernel HIP events)")
    rprof = lat.solve_device(dx, db, KAPPA, CSW, TOL, inner_prec=inner, profile=1)[0]
    k = int(np.argmax(rprof.kernel_ms))
    avg_s = rprof.kernel_ms[k] / rprof.kernel_calls[k] * 1e-3
    achieved = rprof.kernel_bytes[k] / avg_s / 1e9
    po, pv = {"f32": ("P32", "P32"), "f16": ("P16", "P32")}[a.inner]
    symbol = [f"cg_k1<{po}, false>", f"cg_k2<{po}>", f"cg_k1<{po}, true>", f"cg_k4<{po}, {pv}>",
              f"cg_k5<{po}, {pv}>"][k]
    tr = recorded_traffic(symbol)
    result["roofline"] = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
        "frac": round(achieved / 8000.0, 4),
        "traffic": round(tr["bytes_per_launch"] / 1e9, 4) if tr else None,
        "traffic_unit": "GB per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "kernel": f"{symbol} ({KNAMES[k]})",
        "bytes_per_launch": rprof.kernel_bytes[k], "avg_us": round(avg_s * 1e6, 2),
        "launches_timed": rprof.kernel_calls[k],
    }
    if tr:
        result["roofline"]["traffic_source"] = tr["source"]
    result["kernels"] = {
        KNAMES[i]: {"avg_us": round(rprof.kernel_ms[i] / max(1, rprof.kernel_calls[i]) * 1e3, 2),
                    "GB/s": round(rprof.kernel_bytes[i] /
                                  (rprof.kernel_ms[i] / max(1, rprof.kernel_calls[i]) * 1e-3)
                                  / 1e9, 1) if rprof.kernel_ms[i] > 0 else None}
        for i in range(5)}

    log("stand-alone hopping-term sweeps (3 rotated copies) and the copy reference")
    from paper_1103_1363_amd import sweep as _sweep
    copy = _sweep.copy_kernel_rate(lq, torch)
    result["hbm_copy"] = copy
    lats = [lat] + _sweep.make_lattices(lq, dims, 2, u=u, **tiling)
    result["dslash_gbs"] = {p: _sweep.dslash_sweep(lq, lats, torch, p)
                            for p in ("f64", "f32", "f16", "f16x12")}
    for p, d in result["dslash_gbs"].items():
        d["frac_of_copy"] = round(d["GB/s"] / copy["GB/s"], 3)
    del lats
    result["dslash_frac_hbm"] = {p: d["frac_hbm"] for p, d in result["dslash_gbs"].items()}
    log("fused site expressions (SU(3) array products)")
    result["fused_expressions"] = _sweep.su3_sweep(lq, torch, prec=0)
    if not a.no_batched:
        log("12 point sources: batched solve, and one source alone")
        result["batched_12rhs"] = batched_point_sources(lq, lat, torch, dims)
    if not a.no_uneven:
        log("uneven batch of eight lattices: one batch, and one after another")
        result["uneven_batch"] = uneven_batch(lq, torch)
    if not a.no_net:
        log(f"learned preconditioner: {a.net_pairs} training pairs, {a.net_epochs} epochs")
        result["learned_preconditioner"] = learned_preconditioner(lq, lat, torch, db, a.net_pairs,
                                                                  a.net_epochs)

    if not a.no_sap:
        log("SAP-preconditioned FGCR (blocks 8x4x4x4, 3 cycles of 6 MR steps, restart 48) "
            "and SAP-FGMRES-DR (70, 10)")
        result["sap_fgcr"] = sap_fgcr(lq, lat, torch, db, (8, 4, 4, 4), 3, 6, 48)

    log("16^3x32 configuration: FP32 inner iteration against plain FP64")
    result["config_16x16x16x32"] = config_16(lq, torch)

    if not a.no_cpu_baseline:
        log("CPU baseline (oracle)")
        vol = dims[0] * dims[1] * dims[2] * dims[3] / (16 * 16 * 16 * 32)
        its = {"16x16x16x32_plain": (1.0, result["config_16x16x16x32"]["plain_fp64"]["iterations"]),
               "benchmark_plain": (vol, result["plain_fp64"]["iterations"])
               if "plain_fp64" in result else None}
        if "batched_12rhs" in result:
            its["12_point_sources_plain"] = (
                12 * vol, result["batched_12rhs"]["one_source_alone"]["plain_fp64"]["iterations"])
        result["cpu_baseline"] = cpu_baseline(u, b, dims, {k: v for k, v in its.items() if v})
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
