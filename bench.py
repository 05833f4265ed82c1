"""Benchmark of the domain-wall hopping term on one MI355X.

Headline: checkerboarded Dhop at 32^4 x Ls=16 in FP32 (inputs resident in HBM).
One step = one apply in each direction (D^{o<-e} then D^{e<-o}).  Flops are
1320 * Ls per output 4D site per apply; the byte model counts 8 links of 18
reals plus Ls input and Ls output spinors of 24 reals per output 4D site.

Also measured in the same run and reported under "rows": FP64 and 16-bit
Dhop, the Schur normal operator, FP64 vs mixed-precision CG at 24^4 x 12
(time to the FP64 solution), the batched multi-RHS / multi-lattice graph
launch, and the force kernel.  The CPU oracle (plain C, OpenMP) is timed on a
bounded sample of the headline workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--rows all|none|name,...] [--no-cpu]
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

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def dhop_flops(vol, ls, nrhs=1):
    return 1320.0 * ls * (vol // 2) * nrhs


def dhop_bytes(vol, ls, real_bytes, nrhs=1):
    return (8 * 18 + nrhs * ls * 48) * real_bytes * (vol // 2)


def timed(fn, reps, torch):
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    e.synchronize()
    return s.elapsed_time(e) / reps  # ms


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
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
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
    fin = {p: (op.pack(psi_d, 0, p), op.pack(psi_d, 1, p)) for p in ("f32",)}
    fout = {p: (op.field(p), op.field(p)) for p in ("f32",)}
    del psi_d
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
    torch.cuda.synchronize()
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

    # ---------------- plain copy of known size (bandwidth and counter calibration) ----------------
    nbytes = 1 << 30
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    copy_ms = timed(lambda: dst.copy_(src), 10, torch)
    copy_gbs = 2 * nbytes / (copy_ms * 1e-3) / 1e9
    log(f"copy 1 GiB -> 1 GiB: {copy_ms * 1e3:.1f} us, {copy_gbs:.0f} GB/s (read+write)")
    del src, dst
    torch.cuda.empty_cache()

    # ---------------- secondary rows ----------------
    def dhop_row(prec, rb):
        fin[prec] = (op.pack(torch.from_numpy(psi).cuda(), 0, prec), op.pack(torch.from_numpy(psi).cuda(), 1, prec))
        fout[prec] = (op.field(prec), op.field(prec))
        for _ in range(3):
            step(prec)
        ms = timed(lambda: step(prec), 20, torch) / 2
        del fin[prec], fout[prec]
        torch.cuda.empty_cache()
        return {"us_per_apply": ms * 1e3, "gflops": flops / (ms * 1e-3) / 1e9,
                "gbs": dhop_bytes(vol, ls, rb) / (ms * 1e-3) / 1e9,
                "frac_hbm": dhop_bytes(vol, ls, rb) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}

    for prec, rb in (("f64", 8), ("f16", 2), ("bf16", 2)):
        if row_on(f"dhop_32^4x16_{prec}"):
            rows[f"dhop_32^4x16_{prec}"] = dhop_row(prec, rb)
            log(f"row dhop {prec}: {rows[f'dhop_32^4x16_{prec}']}")

    if row_on("mdagm_32^4x16_f32"):
        pin = op.pack(torch.from_numpy(psi).cuda(), 1, "f32")
        out = op.field("f32")
        for _ in range(3):
            D.dwf_mdagm(op.handle, out, pin, "f32")
        ms = timed(lambda: D.dwf_mdagm(op.handle, out, pin, "f32"), 10, torch)
        rows["mdagm_32^4x16_f32"] = {"ms": ms, "dhop_gflops": 4 * flops / (ms * 1e-3) / 1e9}
        log(f"row mdagm: {rows['mdagm_32^4x16_f32']}")
        del pin, out

    # ---------------- CPU oracle baseline ----------------
    cpu = None
    if not args.no_cpu:
        from oracle import coracle as C

        nthreads = C.num_threads()
        # size the sample from a short probe so the run stays within ~cpu-seconds
        probe = 512
        t = time.time()
        C.dhop_cb(u, psi, 1, 0, rows=(0, probe))
        dt = max(time.time() - t, 1e-3)
        nrow = int(min(vol // 2, max(probe, probe * args.cpu_seconds / dt)))
        t = time.time()
        C.dhop_cb(u, psi, 1, 0, rows=(0, nrow))
        dt = time.time() - t
        cpu = {"value": 1320.0 * ls * nrow / dt / 1e9, "unit": "GFlop/s", "cores": nthreads, "kind": "oracle",
               "sample": f"plain C FP64 Dhop_cb on the 32^4x16 input, first {nrow} of {vol // 2} output rows "
                         f"({dt:.1f} s)"}
        log(f"cpu oracle: {cpu}")

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
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_dhop<F32,F32,0,EPI_SCALE>", "algorithmic_bytes_per_launch": algo_bytes,
                     "us_per_launch": round(apply_ms * 1e3, 2)},
        "parity_rel_l2_sampled": parity_err,
        "copy_gbs": round(copy_gbs, 1),
        "frac_of_copy": round(achieved / copy_gbs, 4),
        "cpu_baseline": cpu,
        "rows": rows,
    }
    print(json.dumps(out), flush=True)
    op.close()


if __name__ == "__main__":
    main()
