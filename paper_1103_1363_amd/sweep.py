"""Stand-alone sweeps of the hopping term and the streaming-copy reference,
for bandwidth measurement and for profiling with rocprofv3.

Usage: python -m paper_1103_1363_amd.sweep [--dims 32,32,32,64] [--copies 3]
                                           [--prec f64,f32,f16,f16x12]
                                           [--reps 50] [--copy-kernel]

Each sweep applies H_eo (odd -> even) to `copies` independent (gauge field,
input, output) sets in rotation, so that the working set is several times
the 256 MB Infinity Cache and every launch streams its operands from HBM.
Times come from events on the stream the library launches on.  Algorithmic
bytes per output site: FP64 1152, FP32 576, FP16 296 (12-real links, one
input and one output spinor, FP16 with its 4-byte scale); the 12-RHS FP16
form 8 x 24 + 12 x 104.  Prints one JSON object.
"""
from __future__ import annotations

import argparse
import json
import sys

BYTES = {"f64": 1152, "f32": 576, "f16": 296}


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def dslash_sweep(lq, lats, torch, prec_name, reps=50, warm=5, nrhs=12):
    """Median-free mean time per launch over `reps` launches rotating over the
    lattices' own fields (lats: contexts with their gauge fields uploaded)."""
    import numpy as np
    vh = lats[0].volume // 2
    multi = prec_name == "f16x12"
    prec = {"f64": lq.F64, "f32": lq.F32, "f16": lq.F16, "f16x12": lq.F16X}[prec_name]
    rng = np.random.default_rng(11)
    sets = []
    for lat in lats:
        if multi:
            o = (rng.standard_normal((nrhs, vh, 4, 3))
                 + 1j * rng.standard_normal((nrhs, vh, 4, 3))) / np.sqrt(2)
            din = lat.to_device(o, lq.ODD, prec)
            dout = lat.new_field(lq.EVEN, prec, nrhs)
        else:
            o = (rng.standard_normal((vh, 4, 3)) + 1j * rng.standard_normal((vh, 4, 3))) / np.sqrt(2)
            din = lat.to_device(o, lq.ODD, prec)
            dout = lat.new_field(lq.EVEN, prec)
        sets.append((lat, din, dout))

    def launch(i):
        lat, din, dout = sets[i % len(sets)]
        if multi:
            lat.dslash(dout, din, lq.EVEN, False, prec, nrhs)
        else:
            lat.dslash(dout, din, lq.EVEN, False, prec)

    for i in range(warm):
        launch(i)
    # an event pair around every launch: the sum is kernel time only, without
    # the host's launch gaps between calls
    ev = [_events(torch) for _ in range(reps)]
    torch.cuda.synchronize()
    for i in range(reps):
        ev[i][0].record()
        launch(i)
        ev[i][1].record()
    torch.cuda.synchronize()
    us = sum(a.elapsed_time(b) for a, b in ev) * 1e3 / reps
    per_site = 8 * 24 + nrhs * 104 if multi else BYTES[prec_name]
    gbs = per_site * vh / (us * 1e-6) / 1e9
    flops = 1320 * vh * (nrhs if multi else 1)
    out = {"us": round(us, 2), "bytes_per_site": per_site, "GB/s": round(gbs, 1),
           "frac_hbm": round(gbs / 8000.0, 4), "GFLOP/s": round(flops / (us * 1e-6) / 1e9, 1),
           "copies": len(sets),
           "working_set_GB": round(len(sets) * per_site * vh / 1e9, 3)}
    if multi:
        out["nrhs"] = nrhs
    del sets
    return out


def copy_kernel_rate(lq, torch, nbytes=1 << 30, reps=20):
    """The library's own 16-byte-per-lane streaming copy (lq_stream_copy) of
    nbytes: the achievable HBM bandwidth, read + write."""
    import ctypes as ct
    L = lq.lib()
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)

    def go():
        rc = L.lq_stream_copy(ct.c_void_p(dst.data_ptr()), ct.c_void_p(src.data_ptr()),
                              ct.c_size_t(nbytes), ct.c_void_p(torch.cuda.current_stream().cuda_stream))
        if rc != 0:
            raise RuntimeError(f"lq_stream_copy failed ({rc})")

    for _ in range(3):
        go()
    a, b = _events(torch)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        go()
    b.record()
    torch.cuda.synchronize()
    s = a.elapsed_time(b) * 1e-3 / reps
    assert bool((dst[:4096] == 1).all()) and bool((dst[-4096:] == 1).all())
    del src, dst
    return {"bytes_per_copy": 2 * nbytes, "us": round(s * 1e6, 1),
            "GB/s": round(2 * nbytes / s / 1e9, 1), "kernel": "lq_stream_copy (16 B per lane)"}


def su3_sweep(lq, torch, n=1 << 23, prec=0, reps=20):
    """lq_su3_mul (eq. su3vecmul, U = V W) on n matrices, and the three-factor
    product U = V W X once fused (one pass, 576 B per element in FP64) and once
    as two products (864 B): algorithmic bytes 432 per element for V W."""
    import numpy as np
    cb = 16 if prec == 0 else 8
    nb = lq.site_array_bytes(n, lq.SITE_SU3, prec)
    bufs = [torch.empty(nb, dtype=torch.uint8, device="cuda") for _ in range(5)]
    rng = np.random.default_rng(3)
    small = rng.standard_normal((64, 3, 3)) + 1j * rng.standard_normal((64, 3, 3))
    for b in bufs:  # fill with finite values: tile a small block
        blk = lq.site_array_to_device(small, lq.SITE_SU3, prec)
        b.view(-1)[: blk.numel() * (nb // blk.numel())] = blk.repeat(nb // blk.numel())
    u, v, w, x, t = bufs

    def timed(fn):
        for _ in range(3):
            fn()
        ev = [_events(torch) for _ in range(reps)]
        torch.cuda.synchronize()
        for a, b in ev:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        return sum(a.elapsed_time(b) for a, b in ev) * 1e3 / reps

    us_vw = timed(lambda: lq.su3_mul(u, v, w, n, lq.SU3_VW, prec))
    us_vwx = timed(lambda: lq.su3_mul(u, v, w, n, lq.SU3_VWX, prec, x=x))
    us_two = timed(lambda: (lq.su3_mul(t, v, w, n, lq.SU3_VW, prec),
                            lq.su3_mul(u, t, x, n, lq.SU3_VW, prec)))
    b1 = 27 * cb
    out = {"n": n, "prec": "f64" if prec == 0 else "f32",
           "vw": {"us": round(us_vw, 2), "bytes_per_element": b1,
                  "GB/s": round(b1 * n / (us_vw * 1e-6) / 1e9, 1)},
           "vwx_fused": {"us": round(us_vwx, 2), "bytes_per_element": 36 * cb,
                         "GB/s": round(36 * cb * n / (us_vwx * 1e-6) / 1e9, 1)},
           "vwx_two_passes": {"us": round(us_two, 2), "bytes_per_element": 54 * cb,
                              "GB/s": round(54 * cb * n / (us_two * 1e-6) / 1e9, 1)}}
    out["fused_speedup"] = round(us_two / us_vwx, 3)
    del bufs
    return out


def sap_sweep(lq, torch, lat, block=(8, 4, 4, 4), ncycles=3, nmr=6, reps=5):
    """One SAP application (lq_sap_apply) on a Gaussian FP32 source with each
    block solver: FP32 operator (links in LDS, clover from HBM), FP16
    operator staged in LDS, and the even-odd reduced block solve on the
    FP16 staged operator; mean time over `reps` after one warm-up."""
    from gen import fields
    e = lat.to_device(fields.gaussian_spinor(lat.dims, fields.SEED_SOURCE + 2), lq.FULL, lq.F32)
    y = lat.new_field(lq.FULL, lq.F32)
    out = {"block": list(block), "ncycles": ncycles, "nmr": nmr}
    for name, fp16, eo in (("fp32", False, False), ("fp16_staged", True, False),
                           ("fp16_even_odd", True, True)):
        lat.sap_apply(y, e, block, ncycles, nmr, block_fp16=fp16, block_eo=eo)
        a, b = _events(torch)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            lat.sap_apply(y, e, block, ncycles, nmr, block_fp16=fp16, block_eo=eo)
        b.record()
        torch.cuda.synchronize()
        out[name] = {"ms": round(a.elapsed_time(b) / reps, 3)}
    return out


def make_lattices(lq, dims, copies, seed=1100, u=None, tile_sites=0, mr_tile_sites=0):
    """`copies` contexts, each with its own device copy of one smooth gauge
    field (distinct buffers are what the rotation needs; the values may
    repeat), in the given tiling (0: the library's default)."""
    from gen import fields
    if u is None:
        u = fields.gauge_field(dims, "smooth", seed)
    lats = []
    for _ in range(copies):
        lat = lq.Lattice(dims, tile_sites=tile_sites, mr_tile_sites=mr_tile_sites)
        lat.upload_gauge(u)
        lats.append(lat)
    return lats


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", default="32,32,32,64")
    ap.add_argument("--copies", type=int, default=3)
    ap.add_argument("--prec", default="f64,f32,f16,f16x12")
    ap.add_argument("--reps", type=int, default=50)
    ap.add_argument("--copy-kernel", action="store_true")
    ap.add_argument("--su3", action="store_true", help="the SU(3) array-product sweeps")
    ap.add_argument("--sap", action="store_true",
                    help="one SAP application per block solver (kappa 0.135, csw 1)")
    ap.add_argument("--gauge-cache", default=None,
                    help="an .npy file holding the smooth gauge field (written if absent)")
    a = ap.parse_args()
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch

    from paper_1103_1363_amd import lq
    dims = tuple(int(x) for x in a.dims.split(","))
    out = {"dims": list(dims)}
    if a.copy_kernel:
        out["copy"] = copy_kernel_rate(lq, torch)
    if a.su3:
        out["su3_f64"] = su3_sweep(lq, torch, prec=0)
        out["su3_f32"] = su3_sweep(lq, torch, prec=1)
    precs = [p for p in a.prec.split(",") if p]
    if precs or a.sap:
        print(f"sweep: one gauge field {dims} in {a.copies} contexts", file=sys.stderr, flush=True)
        u = None
        if a.gauge_cache and os.path.exists(a.gauge_cache):
            import numpy as np
            u = np.load(a.gauge_cache)
        elif a.gauge_cache:
            import numpy as np
            from gen import fields
            u = fields.gauge_field(dims, "smooth", 1100)
            np.save(a.gauge_cache, u)
        lats = make_lattices(lq, dims, a.copies, u=u)
        for p in precs:
            print(f"sweep: {p}", file=sys.stderr, flush=True)
            out[p] = dslash_sweep(lq, lats, torch, p, a.reps)
        if a.sap:
            print("sweep: SAP", file=sys.stderr, flush=True)
            lats[0].set_clover(0.135, 1.0)
            out["sap"] = sap_sweep(lq, torch, lats[0])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
