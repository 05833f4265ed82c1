"""Benchmark of the domain-wall fermion hot path on one MI355X.

Headline (the metric's workload): checkerboarded Dhop at 32^4 x Ls=16 in FP32,
inputs resident in HBM.  One step = one apply in each direction
(D^{o<-e} then D^{e<-o}).  Flops are 1320 * Ls per output 4D site per apply;
the byte model counts 8 links of 18 reals plus Ls input and Ls output spinors
of 24 reals per output 4D site.

The other rows of the hot path are measured in the same run and reported
under "rows": FP64 / FP16 / BF16 Dhop, the M5op family, the Schur normal
operator, the FP64 reductions, FP64 vs mixed-precision CG at 24^4 x 12 (time
to the FP64 solution), the batched graph launches, and the force kernel /
differentiable action at 16^4 x 8.  The CPU oracle (plain C, OpenMP) is timed
on a bounded sample of the headline workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--rows all|none|name,...] [--no-cpu]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_2203_06777_amd/csrc/dhop.hip", "paper_2203_06777_amd/csrc/dwf_rows.h",
                  "paper_2203_06777_amd/csrc/dwf_dhop_core.h", "paper_2203_06777_amd/csrc/dwf_device.h",
                  "paper_2203_06777_amd/csrc/dwf_spin.h", "paper_2203_06777_amd/csrc/dwf_common.h",
                  "paper_2203_06777_amd/csrc/dwf_m5inv.h"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def probe_lib():
    """The measurement probes (libdwf_probe.so, built in-tree by __graft_entry__.build())."""
    import ctypes

    path = os.path.join(ROOT, "paper_2203_06777_amd", "libdwf_probe.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    P, U, I = ctypes.c_void_p, ctypes.c_uint, ctypes.c_int
    lib.probe_stream_rows.argtypes = [P, P, P, U, U, U, P]
    lib.probe_link_mult.argtypes = [P, P, P, I, I, I, P]
    lib.probe_dhop_pattern.argtypes = [P, P, P, U, U, U, U, I, I, P]
    lib.probe_read.argtypes = [P, P, ctypes.c_size_t, P]
    return lib


def dhop_flops(vol, ls, nrhs=1):
    return 1320.0 * ls * (vol // 2) * nrhs


def dhop_bytes(vol, ls, real_bytes, nrhs=1):
    return (8 * 18 + nrhs * ls * 48) * real_bytes * (vol // 2)


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def kernel_source_sha():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed counter summary, if it was taken on this kernel source."""
    path = os.path.join(ROOT, "profiles", "dhop_32x32x32x32_ls16_f32_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None, None
    if rec.get("src_sha") != kernel_source_sha():
        return None, rec.get("src_sha")
    return rec.get("bytes_per_launch"), rec.get("src_sha")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--rows", default="all")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2203_06777_amd import dwf as D
    from synth import fields as F

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    D.lib()
    rows = {}
    want_rows = None if args.rows == "all" else set(filter(None, args.rows.split(",")))

    def row_on(name):
        return want_rows is None or name in want_rows

    def timed(fn, reps):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            fn()
        e.record()
        e.synchronize()
        return s.elapsed_time(e) / reps  # ms

    # ---------------- headline: Dhop 32^4 x 16 FP32 ----------------
    w = F.WORKLOADS["dhop_32^4x16"]
    dims, ls = w["dims"], w["ls"]
    vol = int(np.prod(dims))
    t0 = time.time()
    u = F.gauge_field(dims, w["eps"], w["seed_u"])
    psi = F.fermion_cb(dims, ls, w["seed_psi"])
    log(f"generated 32^4x16 inputs in {time.time() - t0:.1f}s")
    op = D.Context(dims, ls, w["M5"], w["mf"])
    op.set_gauge(torch.from_numpy(u).cuda())
    psi_d = torch.from_numpy(psi).cuda()
    fin = {"f32": (op.pack(psi_d, 0, "f32"), op.pack(psi_d, 1, "f32"))}
    fout = {"f32": (op.field("f32"), op.field("f32"))}
    torch.cuda.synchronize()

    def step(prec="f32"):
        ie, io = fin[prec]
        oe, oo = fout[prec]
        D.dwf_dhop(op.handle, oo, ie, 1, 0, prec)
        D.dwf_dhop(op.handle, oe, io, 0, 0, prec)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(args.steps):
        step()
    end.record()
    torch.cuda.synchronize()
    ms_step = start.elapsed_time(end) / args.steps
    apply_ms = ms_step / 2
    flops = dhop_flops(vol, ls)
    gflops = 2 * flops / (ms_step * 1e-3) / 1e9
    algo_bytes = dhop_bytes(vol, ls, 4)
    achieved = algo_bytes / (apply_ms * 1e-3) / 1e9
    log(f"Dhop 32^4x16 f32: {apply_ms * 1e3:.1f} us/apply, {gflops:.0f} GFlop/s, {achieved:.0f} GB/s")

    # sampled parity of the timed output against the oracle
    from oracle import dwf_ref as R

    rng = np.random.default_rng(1)
    rows_s = rng.integers(0, vol // 2, 256)
    got = op.unpack(fout["f32"][1], 1, "f32")[torch.from_numpy(rows_s).cuda()].cpu().numpy()
    want = R.dhop_sites(u, psi, 1, rows_s)
    parity_err = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    log(f"sampled parity rel-L2 {parity_err:.2e}")

    # ---------------- plain copy of known size (bandwidth reference) ----------------
    nbytes = 1 << 30
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    copy_ms = timed(lambda: dst.copy_(src), 10)
    copy_gbs = 2 * nbytes / (copy_ms * 1e-3) / 1e9
    log(f"copy 1 GiB -> 1 GiB: {copy_ms * 1e3:.1f} us, {copy_gbs:.0f} GB/s (read+write)")
    del src, dst
    torch.cuda.empty_cache()

    # ---------------- the apply's compulsory traffic alone (achievable-bandwidth reference) ----------------
    probe = probe_lib()
    nrows = vol // dims[0]
    vx, vl = (dims[0] // 2) * ls * 96 // 16, (dims[0] // 2) * 8 * 18 * 4 // 16  # 16-byte vectors per row
    s_in = torch.empty(nrows * vx * 16, dtype=torch.uint8, device="cuda").fill_(3)
    s_out = torch.empty_like(s_in)
    s_lk = torch.empty(nrows * vl * 16, dtype=torch.uint8, device="cuda").fill_(5)
    cstream = torch.cuda.current_stream().cuda_stream

    def stream_apply():
        rc = probe.probe_stream_rows(s_out.data_ptr(), s_in.data_ptr(), s_lk.data_ptr(), nrows, vx, vl, cstream)
        assert rc == 0, rc

    for _ in range(3):
        stream_apply()
    stream_ms = timed(stream_apply, 20)
    stream_gbs = algo_bytes / (stream_ms * 1e-3) / 1e9
    log(f"compulsory-traffic stream of one apply: {stream_ms * 1e3:.1f} us, {stream_gbs:.0f} GB/s")
    del s_in, s_out, s_lk
    torch.cuda.empty_cache()

    # ---------------- the kernel's memory accesses alone, and re-read bandwidth by footprint ----------------
    if row_on("memory_pattern_32^4x16") and dims == (32, 32, 32, 32) and ls == 16:
        ty_, tz_, tt_ = 8, 4, 32  # the default traversal tile at this shape
        p_in = torch.empty(nrows * vx * 16, dtype=torch.uint8, device="cuda").fill_(3)
        p_out = torch.empty_like(p_in)
        p_lk = torch.empty(nrows * vl * 16, dtype=torch.uint8, device="cuda").fill_(5)
        pat = {}
        for nbr, sto, nm in ((1, 1, "all_accesses"), (0, 1, "no_neighbour_reads"), (1, 0, "no_output_stores")):
            def go():
                assert probe.probe_dhop_pattern(p_out.data_ptr(), p_in.data_ptr(), p_lk.data_ptr(), 32, ty_, tz_, tt_,
                                                nbr, sto, cstream) == 0
            go()
            pat[nm + "_us"] = round(timed(go, 10) * 1e3, 1)
        reads = {}
        sink = torch.empty(16, dtype=torch.uint8, device="cuda")
        for mb in (16, 64, 128, 256, 768):
            nv = mb * (1 << 20) // 16
            t_ms = timed(lambda: probe.probe_read(p_in.data_ptr(), sink.data_ptr(), nv, cstream), 10)
            reads[f"{mb}MB_tbs"] = round(mb * (1 << 20) / (t_ms * 1e-3) / 1e12, 2)
        pat["reread_bandwidth_by_footprint"] = reads
        pat["note"] = ("the row kernel's reads and writes at this shape with no arithmetic (probe_dhop_pattern, tile "
                       f"{ty_}x{tz_}x{tt_}); reread: a grid-stride read of the first N MB over and over")
        rows["memory_pattern_32^4x16"] = pat
        log(f"row memory_pattern: {pat}")
        del p_in, p_out, p_lk
        torch.cuda.empty_cache()

    # ---------------- a1: Dhop in the other precisions ----------------
    def dhop_row(prec, rb):
        fin[prec] = (op.pack(psi_d, 0, prec), op.pack(psi_d, 1, prec))
        fout[prec] = (op.field(prec), op.field(prec))
        for _ in range(3):
            step(prec)
        ms = timed(lambda: step(prec), 20) / 2
        got = op.unpack(fout[prec][1], 1, prec)[torch.from_numpy(rows_s).cuda()].cpu().numpy()
        err = float(np.linalg.norm(got - want) / np.linalg.norm(want))
        del fin[prec], fout[prec]
        torch.cuda.empty_cache()
        gbs = dhop_bytes(vol, ls, rb) / (ms * 1e-3) / 1e9
        return {"us_per_apply": round(ms * 1e3, 1), "gflops": round(flops / (ms * 1e-3) / 1e9, 1),
                "gbs": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4), "rel_l2_vs_oracle": err}

    for prec, rb in (("f64", 8), ("f16", 2), ("bf16", 2)):
        name = f"dhop_32^4x16_{prec}"
        if row_on(name):
            rows[name] = dhop_row(prec, rb)
            log(f"row {name}: {rows[name]}")

    # ---------------- domain decomposition at the headline shape, FP32 ----------------
    if row_on("dd_32^4x16_f32"):
        ie, io = fin["f32"]
        oe, oo = fout["f32"]
        ref = op.field("f32")
        D.dwf_dhop(op.handle, ref, ie, 1, 0, "f32")
        ms_plain = timed(step, 20) / 2
        res = {"plain_us": round(ms_plain * 1e3, 1)}
        for cuts in ("t", "xyz"):
            dd = D.dwf_dd_create(op.handle, "f32", cuts)
            D.dwf_dd_dhop(dd, oo, ie, 1, 0)
            torch.cuda.synchronize()
            same = bool(torch.equal(oo, ref))

            def dd_step():
                D.dwf_dd_dhop(dd, oo, ie, 1, 0)
                D.dwf_dd_dhop(dd, oe, io, 0, 0)

            for _ in range(3):
                dd_step()
            ms_dd = timed(dd_step, 20) / 2
            ms_face = timed(lambda: D.dwf_dd_faces(dd, ie, 1, 0), 20)
            nsites = sum(vol // 2 // dims[mu] for mu in range(4) if "xyzt"[mu] in cuts) * 2
            face_bytes = nsites * ls * (24 + 12) * 4  # slices read, half-spinor faces written
            res[f"cut_{cuts}"] = {
                "decomposed_us": round(ms_dd * 1e3, 1), "overhead": round(ms_dd / ms_plain - 1.0, 3),
                "faces": nsites // (vol // 2 // dims[3]), "face_mb_total": round(nsites * ls * 12 * 4 / 1e6, 1),
                "face_assembly_us": round(ms_face * 1e3, 1),
                "face_assembly_gbs": round(face_bytes / (ms_face * 1e-3) / 1e9, 1),
                "bitwise_equal_to_dhop": same}
            D.dwf_dd_destroy(dd)
        rows["dd_32^4x16_f32"] = res
        log(f"row dd: {res}")

    # ---------------- a2/a3/a4 at the headline shape, FP32 ----------------
    if row_on("m5_mdagm_blas_32^4x16_f32"):
        x = fin["f32"][1]
        y = op.field("f32")
        cbb = dhop_bytes(vol, ls, 4) - 8 * 18 * 4 * (vol // 2)  # one field in + one out
        r = {}
        for nm, dag, inv in (("m5", 0, 0), ("m5inv", 0, 1), ("m5inv_dag", 1, 1)):
            ms = timed(lambda: D.dwf_m5(op.handle, y, x, dag, inv, 0, "f32"), 20)
            r[nm] = {"us": round(ms * 1e3, 1), "gbs": round(cbb / (ms * 1e-3) / 1e9, 1)}
        ms = timed(lambda: D.dwf_mdagm(op.handle, y, x, "f32"), 10)
        r["mdagm"] = {"ms": round(ms, 3), "dhop_gflops": round(4 * flops / (ms * 1e-3) / 1e9, 1)}
        ms = timed(lambda: D.dwf_norm2(op.handle, x, 0, "f32"), 20)
        r["norm2_sync"] = {"us": round(ms * 1e3, 1), "gbs": round(cbb / 2 / (ms * 1e-3) / 1e9, 1)}
        ms = timed(lambda: D.dwf_axpy(op.handle, y, 0.5, x, 0, "f32"), 20)
        r["axpy"] = {"us": round(ms * 1e3, 1), "gbs": round(1.5 * cbb / (ms * 1e-3) / 1e9, 1)}
        rows["m5_mdagm_blas_32^4x16_f32"] = r
        log(f"row m5/mdagm/blas: {r}")
        del y
    del psi_d, fin, fout
    torch.cuda.empty_cache()

    # ---------------- CPU oracle baseline (bounded sample of the headline workload) ----------------
    cpu = None
    if not args.no_cpu:
        from oracle import coracle as C

        nthreads = C.num_threads()
        C.dhop_cb(u, psi, 1, 0, rows=(0, 4096))  # warm-up (threads, first-touch pages)
        # whole applies of the oracle (each call as it stands) until about cpu_seconds have passed
        nrow, passes = vol // 2, 0
        t = time.time()
        while passes == 0 or time.time() - t < args.cpu_seconds:
            C.dhop_cb(u, psi, 1, 0)
            passes += 1
        dt = time.time() - t
        cpu = {"value": round(1320.0 * ls * nrow * passes / dt / 1e9, 3), "unit": "GFlop/s", "cores": nthreads,
               "kind": "oracle",
               "sample": f"plain C FP64 Dhop_cb (oracle) on the 32^4x16 input: {passes} whole applies "
                         f"({nrow} output rows each), {dt:.1f} s",
               "host_cpu": host_cpu_model()}
        # one core: a contiguous slice of the output rows of the same apply
        C.set_num_threads(1)
        nsl = nrow // 16
        t = time.time()
        C.dhop_cb(u, psi, 1, 0, rows=(0, nsl))
        dt1 = time.time() - t
        C.set_num_threads(nthreads)
        cpu["one_core"] = {"value": round(1320.0 * ls * nsl / dt1 / 1e9, 3), "unit": "GFlop/s",
                           "sample": f"{nsl} output rows of the 32^4x16 apply, {dt1:.1f} s"}
        log(f"cpu oracle: {cpu}")
    op.close()
    del u, psi
    if cpu is not None:
        # the other oracle timings of the hot path: 16^4 x 16 Dhop_cb and the 24^4 x 12 normal operator
        w16 = F.WORKLOADS["dhop_16^4x16"]
        u16 = F.gauge_field(w16["dims"], w16["eps"], w16["seed_u"])
        p16 = F.fermion_cb(w16["dims"], w16["ls"], w16["seed_psi"])
        reps, t = 0, time.time()
        while reps < 3 or time.time() - t < 3.0:
            C.dhop_cb(u16, p16, 1, 0)
            reps += 1
        dt16 = (time.time() - t) / reps
        cpu["dhop_16^4x16"] = {"value": round(1320.0 * w16["ls"] * (16 ** 4 // 2) / dt16 / 1e9, 3),
                               "unit": "GFlop/s", "sample": f"{reps} whole applies"}
        del u16, p16
        wc = F.WORKLOADS["cg_24^4x12"]
        uc = F.gauge_field(wc["dims"], wc["eps"], wc["seed_u"])
        bc = F.fermion_cb(wc["dims"], wc["ls"], wc["seed_psi"])
        t = time.time()
        C.mdagm(uc, bc, wc["M5"], wc["mf"])
        dtm = time.time() - t
        cpu["mdagm_24^4x12"] = {"seconds": round(dtm, 3),
                                "note": "one M_pc^dag M_pc (4 Dhop_cb + M5op terms); a CG iteration is this plus "
                                        "three vector passes, so FP64 CG to 1e-10 costs about iterations x this"}
        del uc, bc
        log(f"cpu oracle (other workloads): 16^4x16 {cpu['dhop_16^4x16']}, mdagm {cpu['mdagm_24^4x12']}")

    # ---------------- a5/a6: FP64 vs mixed CG at 24^4 x 12 ----------------
    if row_on("cg_24^4x12"):
        w = F.WORKLOADS["cg_24^4x12"]
        cdims, cls = w["dims"], w["ls"]
        u2 = F.gauge_field(cdims, w["eps"], w["seed_u"])
        b = F.fermion_cb(cdims, cls, w["seed_psi"])
        op2 = D.Context(cdims, cls, w["M5"], w["mf"])
        op2.set_gauge(torch.from_numpy(u2).cuda())
        bi = op2.pack(torch.from_numpy(b).cuda(), 1, "f64")
        # launch shapes from the autotuner for every operator precision, outside the timed solves
        tuned = {}
        for prec in ("f64", "f32", "f16", "bf16"):
            for dag in (0, 1):
                tuned[f"{prec}/{dag}"] = round(D.dwf_tune(op2.handle, prec, dag), 1)
        log(f"cg tuned dhop us: {tuned}")
        sol = {}
        r = {"tuned_dhop_us": tuned}
        for mode in range(4):  # warm-up: workspace allocation and first launches
            D.dwf_cg(op2.handle, op2.zeros("f64"), bi, 1e-2, 50000, mode)
        for mode, nm in ((0, "fp64"), (1, "mixed_fp32"), (2, "mixed_fp16"), (3, "mixed_bf16")):
            x = op2.zeros("f64")
            torch.cuda.synchronize()
            t = time.time()
            st = D.dwf_cg(op2.handle, x, bi, w["tol"], 50000, mode)
            torch.cuda.synchronize()
            wall = time.time() - t
            sol[mode] = x
            r[nm] = {"seconds": round(wall, 4), "iters": st["inner_iters"], "outer": st["outer_iters"],
                     "true_rel_resid": st["true_rel_resid"]}
        nref = D.dwf_norm2(op2.handle, sol[0], 0, "f64")
        for mode, nm in ((1, "mixed_fp32"), (2, "mixed_fp16"), (3, "mixed_bf16")):
            d = op2.field("f64")
            d.copy_(sol[mode])
            D.dwf_axpy(op2.handle, d, -1.0, sol[0], 0, "f64")
            r[nm]["rel_l2_vs_fp64"] = float(np.sqrt(D.dwf_norm2(op2.handle, d, 0, "f64") / nref))
            r[nm]["speedup_vs_fp64"] = round(r["fp64"]["seconds"] / r[nm]["seconds"], 3)
        rows["cg_24^4x12"] = r
        log(f"row cg: {r}")

        # Moebius (Cayley) operator, b = 1.5, c = 0.5, on the same lattice, gauge and right-hand side
        if row_on("mobius_24^4x12"):
            rm = {"b": 1.5, "c": 0.5}
            tmp = op2.field("f32")
            p32 = op2.field("f32")
            D.dwf_convert(op2.handle, p32, "f32", bi, "f64", 0)
            rm["shamir_mdagm_f32_us"] = round(timed(lambda: D.dwf_mdagm(op2.handle, tmp, p32, "f32"), 20) * 1e3, 1)
            op2.set_mobius(1.5, 0.5)
            rm["mobius_mdagm_f32_us"] = round(timed(lambda: D.dwf_mdagm(op2.handle, tmp, p32, "f32"), 20) * 1e3, 1)
            msol = {}
            for mode in (0, 2):
                D.dwf_cg(op2.handle, op2.zeros("f64"), bi, 1e-2, 50000, mode)
            for mode, nm in ((0, "fp64"), (2, "mixed_fp16")):
                x = op2.zeros("f64")
                torch.cuda.synchronize()
                t = time.time()
                st = D.dwf_cg(op2.handle, x, bi, w["tol"], 50000, mode)
                torch.cuda.synchronize()
                msol[mode] = x
                rm[nm] = {"seconds": round(time.time() - t, 4), "iters": st["inner_iters"], "outer": st["outer_iters"],
                          "true_rel_resid": st["true_rel_resid"]}
            d = op2.field("f64")
            d.copy_(msol[2])
            D.dwf_axpy(op2.handle, d, -1.0, msol[0], 0, "f64")
            rm["mixed_fp16"]["rel_l2_vs_fp64"] = float(
                np.sqrt(D.dwf_norm2(op2.handle, d, 0, "f64") / D.dwf_norm2(op2.handle, msol[0], 0, "f64")))
            rm["mixed_fp16"]["speedup_vs_fp64"] = round(rm["fp64"]["seconds"] / rm["mixed_fp16"]["seconds"], 3)
            rows["mobius_24^4x12"] = rm
            log(f"row mobius: {rm}")
        op2.close()
        del sol, bi, u2, b
        torch.cuda.empty_cache()

    # ---------------- a7: batched graph launches ----------------
    if row_on("batched"):
        r = {}

        def same_as_singles(handles, ins, outs, nrhs):
            """Every batched output equals the single-field dwf_dhop of the same input bit for bit."""
            k, ok = 0, True
            for li, h in enumerate(handles):
                for _ in range(nrhs[li]):
                    single = torch.empty_like(outs[k])
                    D.dwf_dhop(h, single, ins[k], 0, 0, "f32")
                    ok = ok and bool(torch.equal(single, outs[k]))
                    k += 1
            return ok

        w = F.WORKLOADS["batch_32^4x12x12"]
        bdims, bls = w["dims"], w["ls"]
        op3 = D.Context(bdims, bls, w["M5"], w["mf"])
        op3.set_gauge(torch.from_numpy(F.gauge_field(bdims, w["eps"], w["seed_u"])).cuda())
        nr = len(w["rhs_seeds"])
        ins, outs = [], []
        for sd in w["rhs_seeds"]:  # the workload's seeds, 2040 + r
            ins.append(op3.pack(torch.from_numpy(F.fermion_cb(bdims, bls, sd)).cuda(), 1, "f32"))
            outs.append(op3.field("f32"))
        plan = D.dwf_batch_plan([op3.handle], [nr], "f32", 0)
        D.dwf_batch_capture(plan, outs, ins, 0)
        for _ in range(2):
            D.dwf_batch_launch(plan)
        ms = timed(lambda: D.dwf_batch_launch(plan), 5)
        torch.cuda.synchronize()
        same = same_as_singles([op3.handle], ins, outs, [nr])
        ms1 = timed(lambda: [D.dwf_dhop(op3.handle, outs[k], ins[k], 0, 0, "f32") for k in range(nr)], 3)
        fl = dhop_flops(vol, bls, nr)
        by = dhop_bytes(vol, bls, 4, nr)
        r["32^4x12x12rhs"] = {"graph_ms": round(ms, 3), "gflops": round(fl / (ms * 1e-3) / 1e9, 1),
                               "gbs": round(by / (ms * 1e-3) / 1e9, 1), "frac_hbm": round(by / (ms * 1e-3) / 8e12, 3),
                               "per_rhs_launches_ms": round(ms1, 3), "bitwise_equal_to_single_applies": same}
        D.dwf_batch_free(plan)
        del ins, outs
        op3.close()
        torch.cuda.empty_cache()
        wm = F.WORKLOADS["batch_mixed"]
        ctxs, ins, outs, nrhs = [], [], [], []
        fl = by = 0.0
        for lat in wm["lattices"]:
            ld, lls = lat["dims"], lat["ls"]
            o = D.Context(ld, lls, wm["M5"], wm["mf"])
            o.set_gauge(torch.from_numpy(F.gauge_field(ld, wm["eps"], lat["seed_u"])).cuda())
            ctxs.append(o)
            nrhs.append(len(lat["rhs_seeds"]))
            v = int(np.prod(ld))
            for sd in lat["rhs_seeds"]:  # seeds 1000 L + r
                ins.append(o.pack(torch.from_numpy(F.fermion_cb(ld, lls, sd)).cuda(), 1, "f32"))
                outs.append(o.field("f32"))
            fl += dhop_flops(v, lls, nrhs[-1])
            by += dhop_bytes(v, lls, 4, nrhs[-1])
        plan = D.dwf_batch_plan([c.handle for c in ctxs], nrhs, "f32", 0)
        D.dwf_batch_capture(plan, outs, ins, 0)
        for _ in range(2):
            D.dwf_batch_launch(plan)
        ms = timed(lambda: D.dwf_batch_launch(plan), 20)

        def singles():
            k = 0
            for li, o in enumerate(ctxs):
                for _ in range(nrhs[li]):
                    D.dwf_dhop(o.handle, outs[k], ins[k], 0, 0, "f32")
                    k += 1

        torch.cuda.synchronize()
        same = same_as_singles([c.handle for c in ctxs], ins, outs, nrhs)
        ms1 = timed(singles, 5)
        r["mixed_8_12_16_20x8x4rhs"] = {"graph_ms": round(ms, 4), "gflops": round(fl / (ms * 1e-3) / 1e9, 1),
                                         "gbs": round(by / (ms * 1e-3) / 1e9, 1), "per_rhs_launches_ms": round(ms1, 4),
                                         "bitwise_equal_to_single_applies": same}
        D.dwf_batch_free(plan)
        for c in ctxs:
            c.close()
        del ins, outs
        torch.cuda.empty_cache()
        rows["batched_f32"] = r
        log(f"row batched: {r}")

    # ---------------- a8: force kernel and differentiable action at 16^4 x 8 ----------------
    if row_on("force_16^4x8"):
        from paper_2203_06777_amd.autograd import dwf_action

        w = F.WORKLOADS["force_16^4x8"]
        fdims, fls = w["dims"], w["ls"]
        op4 = D.Context(fdims, fls, w["M5"], w["mf"])
        U = torch.from_numpy(F.gauge_field(fdims, w["eps"], w["seed_u"])).cuda().requires_grad_(True)
        phi = torch.from_numpy(F.fermion_full(fdims, fls, w["seed_phi"])).cuda()
        torch.cuda.synchronize()
        t = time.time()
        s = dwf_action(op4, U, phi, 1e-10)
        s.backward()
        torch.cuda.synchronize()
        wall = time.time() - t
        X = op4.pack(phi, 2, "f64")
        Y = op4.pack(torch.from_numpy(F.fermion_full(fdims, fls, w["seed_phi"] + 1)).cuda(), 2, "f64")
        Fo = torch.empty_like(U)
        ms = timed(lambda: D.dwf_force(op4.handle, Fo, X, Y, 1, 1.0), 10)
        fv = int(np.prod(fdims))
        # compulsory HBM bytes: X and Y read once, U_mu(x) read and F_mu(x) written once
        fbytes = fv * (2 * 24 * 8 * fls + 2 * 4 * 18 * 8)
        gbs = fbytes / (ms * 1e-3) / 1e9
        rows["force_16^4x8"] = {"action_plus_grad_seconds": round(wall, 3), "force_kernel_us": round(ms * 1e3, 1),
                                "force_kernel_gbs": round(gbs, 1), "force_kernel_frac": round(gbs / HBM_PEAK_GBS, 3)}
        log(f"row force: {rows['force_16^4x8']}")

        # HMC trajectory consuming the force: pseudofermion heatbath, 5 leapfrog steps, Metropolis
        if row_on("hmc_16^4x8"):
            from paper_2203_06777_amd import hmc as HM

            rh = {"eps": 0.002, "nsteps": 5, "solver_tol": 1e-10}  # dH = O(1) on these rough random links
            U0 = U.detach().clone()
            eta = torch.from_numpy(F.fermion_full(fdims, fls, w["seed_phi"] + 2)).cuda()
            P0 = torch.from_numpy(F.su3_directions(fdims, w["seed_phi"] + 3)).cuda()
            phi_h = HM.pseudofermion(op4, U0, eta)
            for mode, nm in ((0, "fp64_solves"), (2, "mixed_fp16_solves")):
                Ut = U0.clone()
                torch.cuda.synchronize()
                t = time.time()
                tr = HM.trajectory(op4, Ut, P0.clone(), phi_h, rh["eps"], rh["nsteps"], 0.5, rh["solver_tol"], mode)
                torch.cuda.synchronize()
                rh[nm] = {"seconds": round(time.time() - t, 3), "dH": tr["dH"], "accepted": tr["accepted"]}
            rows["hmc_16^4x8"] = rh
            log(f"row hmc: {rh}")
        op4.close()

    # ---------------- the link multiply on the vector ALUs and on the matrix cores ----------------
    if row_on("link_mult_probe"):
        rng2 = np.random.default_rng(7)
        u3 = F.gauge_field((2, 2, 2, 2), 0.5, 11)[0, 0, 0, 0, 0]  # one SU(3) matrix
        m6 = np.block([[u3.real, -u3.imag], [u3.imag, u3.real]]).astype(np.float32)  # real form, orthogonal
        mat = torch.from_numpy(m6.ravel().copy()).cuda()
        nwg, reps = 4096, 256
        ncol = {0: nwg * 256, 1: nwg * 64, 2: nwg * 64}
        cols = torch.from_numpy(rng2.standard_normal(nwg * 256 * 6).astype(np.float32)).cuda()
        res = {}
        for mode, nm in ((0, "valu"), (1, "mfma_operands_in_place"), (2, "mfma_with_lane_shuffles")):
            out_t = torch.empty(ncol[mode] * 6, dtype=torch.float32, device="cuda")
            cst = torch.cuda.current_stream().cuda_stream

            def go(r):
                assert probe.probe_link_mult(out_t.data_ptr(), mat.data_ptr(), cols.data_ptr(), mode, nwg, r, cst) == 0

            go(1)  # one product: checked against the CPU
            torch.cuda.synchronize()
            xc = cols[: ncol[mode] * 6].cpu().numpy().reshape(-1, 6).astype(np.float64)
            ref = xc @ m6.astype(np.float64).T
            err = float(np.abs(out_t.cpu().numpy().reshape(-1, 6) - ref).max() / np.abs(ref).max())
            ms = timed(lambda: go(reps), 5)
            tf = ncol[mode] * reps * 72 / (ms * 1e-3) / 1e12
            res[nm] = {"useful_tflops": round(tf, 1), "one_product_max_rel_err": err}
        res["note"] = ("(6x6 real) x (6 x N) link multiply, operands in registers, " f"{nwg} workgroups x {reps} "
                       "rounds; useful flops 72 per column; MFMA = v_mfma_f32_16x16x4f32 on a 16x8 padded matrix")
        rows["link_mult_probe"] = res
        log(f"row link_mult_probe: {res}")

    # ---------------- software-managed device cache: host fields beyond a device budget ----------------
    if row_on("cache_16^4x16_f32"):
        w = F.WORKLOADS["dhop_16^4x16"]
        cdims, cls = w["dims"], w["ls"]
        op5 = D.Context(cdims, cls, w["M5"], w["mf"])
        op5.set_gauge(torch.from_numpy(F.gauge_field(cdims, w["eps"], w["seed_u"])).cuda())
        base = op5.pack(torch.from_numpy(F.fermion_cb(cdims, cls, w["seed_psi"])).cuda(), 0, "f32")
        nb = base.numel()
        nf, slots, rounds = 8, 6, 3  # 8 input + 8 output fields in pinned host memory, device budget 6 fields
        hin, hout = [], []
        for i in range(nf):
            d = (base.view(torch.float32) * (1.0 + 0.125 * i)).view(torch.uint8)
            hin.append(torch.empty(nb, dtype=torch.uint8, pin_memory=True).copy_(d))
            hout.append(torch.zeros(nb, dtype=torch.uint8, pin_memory=True))
        dres_in, dres_out = base.clone(), op5.zeros("f32")
        us_res = timed(lambda: D.dwf_dhop(op5.handle, dres_out, dres_in, 1, 0, "f32"), 20) * 1e3
        h2d_ms = timed(lambda: dres_in.copy_(hin[0], non_blocking=True), 10)
        cache = D.dwf_cache_create(slots * nb, D.DWF_CACHE_DEVICE)

        def sweep():
            for i in range(nf):
                vi = D.dwf_cache_open(cache, hin[i], nb, D.DWF_ACC_READ)
                vo = D.dwf_cache_open(cache, hout[i], nb, D.DWF_ACC_WRITE)
                D.dwf_dhop(op5.handle, vo, vi, 1, 0, "f32")
                D.dwf_cache_close(cache, hin[i])
                D.dwf_cache_close(cache, hout[i])

        sweep()  # fills the budget
        torch.cuda.synchronize()
        s0 = D.dwf_cache_get_stats(cache)
        t = time.time()
        for _ in range(rounds):
            sweep()
        torch.cuda.synchronize()
        wall = time.time() - t
        s1 = D.dwf_cache_get_stats(cache)
        moved = (s1["h2d_bytes"] - s0["h2d_bytes"]) + (s1["d2h_bytes"] - s0["d2h_bytes"])
        D.dwf_cache_open(cache, hout[nf - 1], nb, D.DWF_CPU_READ)
        D.dwf_dhop(op5.handle, dres_out, dres_in.copy_(hin[nf - 1]), 1, 0, "f32")
        same = bool(torch.equal(hout[nf - 1], dres_out.cpu()))
        D.dwf_cache_close(cache, hout[nf - 1])
        D.dwf_cache_destroy(cache)
        rows["cache_16^4x16_f32"] = {
            "fields_bytes": 2 * nf * nb, "device_budget_bytes": slots * nb,
            "us_per_apply_through_cache": round(wall / (rounds * nf) * 1e6, 1),
            "us_per_apply_resident": round(us_res, 1),
            "migrated_gb_per_apply": round(moved / (rounds * nf) / 1e9, 4),
            "migration_gbs": round(moved / wall / 1e9, 1),
            "pinned_h2d_copy_gbs": round(nb / (h2d_ms * 1e-3) / 1e9, 1),
            "evictions": s1["evictions"] - s0["evictions"],
            "bitwise_equal_to_resident_apply": same,
        }
        log(f"row cache: {rows['cache_16^4x16_f32']}")
        del hin, hout, dres_in, dres_out, base
        op5.close()
        torch.cuda.empty_cache()

    traffic, sha = measured_traffic()
    out = {
        "metric": "DWF Dhop GFlop/s & HBM GB/s on 1 GPU; mixed vs FP64 CG time-to-1e-8",
        "value": round(gflops, 1),
        "unit": "GFlop/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded SU(3) links eps=0.5, Gaussian fermions)",
        "config": {"workload": "dhop_cb 32^4 x Ls=16 FP32, one apply per parity per step", "dims": list(dims),
                   "Ls": ls, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     # FETCH_SIZE counts every L2 fill from the fabric, Infinity-Cache hits included:
                     # an upper bound on the HBM bytes
                     "traffic_counts": "L2 fills (FETCH_SIZE) + L2 writes (WRITE_SIZE), calibrated on a 1 GiB copy",
                     "kernel": "k_dhop_rows<F32,F32,0,EPI_SCALE,16>", "algorithmic_bytes_per_launch": algo_bytes,
                     "us_per_launch": round(apply_ms * 1e3, 2), "kernel_src_sha": kernel_source_sha()},
        "parity_rel_l2_sampled": parity_err,
        "copy_gbs": round(copy_gbs, 1),
        "frac_of_copy": round(achieved / copy_gbs, 4),
        # a kernel that moves exactly the apply's compulsory bytes in the same row shape, no arithmetic
        "stream_gbs": round(stream_gbs, 1),
        "frac_of_stream": round(achieved / stream_gbs, 4),
        "cpu_baseline": cpu,
        # the paper's own figures, on other hardware and an unstated workload: context, not the target
        "paper_context": {"dwf_tflops_per_gpu": 1.3, "hardware": "AMD MI100 (early HIP port)",
                          "dwf_kernels_hbm_frac": 0.8, "hardware_bw": "NVIDIA A100",
                          "note": "no lattice size, Ls, precision or byte model stated"},
        "rows": rows,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
