#!/usr/bin/env python3
"""Benchmark of the compression hot path on one MI355X.

One step = compress + decompress of a 513^3 float32 turbulence-like field
(spectral synthesis, E(k) ~ k^-5/3, seed 2) at relative L-infinity tolerance
1e-3: max|u| pass, device bin widths, multilevel decomposition with fused
quantization, histogram, Huffman codebook and encode; then decode, dequantize
and recomposition.  The field and every buffer are resident in HBM before the
timed region; outputs stay on the device.

Prints one JSON line: round-trip throughput (input bytes / step time), the
roofline of the dominant kernel (HIP-event duration on its stream, algorithmic
bytes per launch, HBM peak 8 TB/s) and the CPU oracle timed on a bounded
sample on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "coeff_r21_fine_513cubed_f32_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2401_05994_amd", "csrc", "transform3d.hip")


# The finest decomposition kernel and every device helper it uses come before
# this line of its source file; what follows (other kernels, host code) does
# not change it.
KERNEL_SOURCE_END = b"// mass + restriction along dim 0 of g1"


def source_sha256(path: str) -> str:
    """sha256 of the kernel's source text: the file up to KERNEL_SOURCE_END
    (the whole file if the marker is missing)."""
    import hashlib

    with open(path, "rb") as f:
        text = f.read()
    end = text.find(KERNEL_SOURCE_END)
    return hashlib.sha256(text if end < 0 else text[:end]).hexdigest()


def measured_traffic(n: int, tol: float):
    """HBM bytes per launch of the finest decomposition kernel, from the committed
    counter summary (FETCH_SIZE + WRITE_SIZE, each scaled by a plain copy of known
    size); None when the kernel source has changed since the counters were taken
    or the summary covers another workload."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    fields = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    try:
        if fields["kernel source sha256"] != source_sha256(KERNEL_SOURCE):
            return None
        if int(fields["n"]) != n or float(fields["tol"]) != tol:
            return None
        return int(fields["traffic bytes per launch"])
    except (KeyError, ValueError):
        return None


def algorithmic_bytes(kernel: str, n: int, dtype_bytes: int, levels_sizes):
    """Bytes a kernel must move per launch (each input read once, each output written once)."""
    nf = levels_sizes[-1]
    nc = levels_sizes[-2]
    N = nf ** 3
    Nc = nc ** 3
    s = dtype_bytes
    if kernel == "coeff_r21_fine":
        # the level's own work: read u once; write the new nodes' 2-byte symbols and
        # the coarse copy (the intermediate it also writes is this design's, and is
        # reported separately)
        return N * s + 2 * (N - Nc) + Nc * s
    if kernel == "interp_add3_fine":
        # read the new nodes' symbols and the coarse grid; write u
        return 2 * (N - Nc) + Nc * s + N * s
    if kernel == "scatter_r21_fine":
        # read the new nodes' symbols; write the restricted plane
        return 2 * (N - Nc) + nf * nc * nc * s
    return None


def bench_batch(m, torch, launches: int = 3, tol: float = 1e-3):
    """The 256-field uneven-shape batch (2D 65..2049 per side, 3D 33..257, slopes U[-4, -5/3],
    rel Linf tol 1e-3): plan (tuning + capture) once, then time whole-graph launches."""
    import fieldgen

    specs = fieldgen.batch_specs()
    fields = []
    for i, sp in enumerate(specs):
        # host synthesis: one FFT size per field, which the host does in seconds
        fields.append(torch.from_numpy(fieldgen.spectral(sp.shape, sp.beta, sp.seed).astype("float32")).cuda())
        if (i + 1) % 64 == 0:
            print(f"[bench] batch: generated {i + 1}/{len(specs)} fields", file=sys.stderr, flush=True)
    in_bytes = sum(f.numel() * 4 for f in fields)
    print(f"[bench] batch: {len(fields)} fields, {in_bytes / 1e9:.3f} GB", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    b = m.Batch(fields, tol)
    plan_s = time.perf_counter() - t0
    print(f"[bench] batch: planned (tuning + capture) in {plan_s:.1f} s", file=sys.stderr, flush=True)
    b.launch()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(launches):
        b.launch()
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / launches
    res = b.results()
    out_bytes = sum(sz for _, sz in res)
    # spot check: the largest field decompresses within its bound
    big = max(range(len(fields)), key=lambda i: fields[i].numel())
    rec = m.mgard_decompress(res[big][0], res[big][1])
    err = float((rec - fields[big]).abs().max())
    tau = tol * float(fields[big].abs().max())
    assert err <= tau, f"batch field {big}: L-infinity error {err} exceeds {tau}"
    nk = b.launches
    b.close()
    print(f"[bench] batch: {ms:.2f} ms per launch, {nk} kernel launches per graph (plan {plan_s:.1f} s)",
          file=sys.stderr, flush=True)
    return {"workload": "256 seeded float32 fields of uneven shapes (2D 65..2049 per side, 3D 33..257), "
                        "slopes U[-4,-5/3], rel Linf 1e-3, one graph launch", "fields": len(fields),
            "in_bytes": in_bytes, "ms_per_launch": round(ms, 3), "GBps": round(in_bytes / (ms * 1e-3) / 1e9, 3),
            "ratio": round(in_bytes / out_bytes, 4), "plan_s": round(plan_s, 2), "launches": launches,
            "kernel_launches_per_graph": nk}


def bench_chunked(m, torch, n: int = 1025, slab: int = 129, tol: float = 1e-3, reps: int = 2):
    """Out-of-core path: an n^3 float32 spectral k^-5/3 field (seed 5) in pinned host memory,
    compressed in slabs of `slab` planes and decompressed back to pinned host memory.  The
    times include every host-device copy (PCIe), so this rate is reported beside the
    device-resident metric, never as it."""
    import fieldgen

    print(f"[bench] chunked: generating {n}^3", file=sys.stderr, flush=True)
    ud = fieldgen.spectral((n, n, n), -5.0 / 3.0, 5, device="cuda").to(torch.float32)
    uh = torch.empty(ud.shape, dtype=torch.float32, pin_memory=True)
    uh.copy_(ud)
    del ud
    torch.cuda.empty_cache()
    in_bytes = uh.numel() * 4
    buf, nb = m.mgard_compress_chunked(uh, tol, slab)  # warm-up: tables, scratch
    rec = m.mgard_decompress_chunked(buf, nb)
    tc, td = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        a = time.perf_counter()
        buf, nb = m.mgard_compress_chunked(uh, tol, slab, out=buf)
        torch.cuda.synchronize()
        b = time.perf_counter()
        m.mgard_decompress_chunked(buf, nb, out=rec)
        torch.cuda.synchronize()
        tc.append(b - a)
        td.append(time.perf_counter() - b)
    tau = tol * float(uh.abs().max())
    err = float((rec - uh).abs().max())
    assert err <= tau, f"chunked: L-infinity error {err} exceeds {tau}"
    nsl = len(range(0, n, slab)) - (1 if n % slab and n % slab < 3 and n > slab else 0)
    print(f"[bench] chunked: compress {min(tc) * 1e3:.1f} ms, decompress {min(td) * 1e3:.1f} ms",
          file=sys.stderr, flush=True)
    return {"workload": f"{n}^3 float32 spectral k^-5/3 field (seed 5) in pinned host memory, slabs of {slab} "
                        f"planes, rel Linf tol {tol}, host to host",
            "in_bytes": in_bytes, "slabs": nsl, "compress_ms": round(min(tc) * 1e3, 2),
            "decompress_ms": round(min(td) * 1e3, 2),
            "compress_GBps": round(in_bytes / min(tc) / 1e9, 3), "decompress_GBps": round(in_bytes / min(td) / 1e9, 3),
            "ratio": round(in_bytes / nb, 4), "linf_over_tau": round(err / tau, 4), "includes_pcie": True}


def timed_round_trip(m, torch, u, tol, steps, coords=None, lossless=False, kernels=False):
    """Compress + decompress of a device-resident field: rates, ratio, L-inf / tau and, with
    kernels=True, the decomposition + quantization kernel time per compress (HIP events)."""
    dt = m.F32 if u.dtype == torch.float32 else m.F64
    out = torch.empty(m.mgard_compress_bound(tuple(u.shape), dt, coords), dtype=torch.uint8, device=u.device)
    rec = torch.empty_like(u)
    kw = {} if coords is None else {"coords": coords}
    for _ in range(2):
        buf, nb, info = m.mgard_compress(u, tol, out=out, lossless=lossless, **kw)
        m.mgard_decompress(buf, nb, out=rec)
    torch.cuda.synchronize()
    tc = td = 0.0
    for _ in range(steps):
        a = time.perf_counter()
        buf, nb, info = m.mgard_compress(u, tol, out=out, lossless=lossless, **kw)
        b = time.perf_counter()
        m.mgard_decompress(buf, nb, out=rec)
        torch.cuda.synchronize()
        tc += b - a
        td += time.perf_counter() - b
    in_bytes = u.numel() * u.element_size()
    err = float((rec.double() - u.double()).abs().max())
    tau = info["tau_abs"]
    assert err <= tau, f"L-infinity error {err} exceeds {tau}"
    r = {"ms_round_trip": round((tc + td) / steps * 1e3, 3), "GBps": round(in_bytes * steps / (tc + td) / 1e9, 3),
         "compress_GBps": round(in_bytes * steps / tc / 1e9, 3),
         "decompress_GBps": round(in_bytes * steps / td / 1e9, 3), "ratio": round(in_bytes / nb, 4),
         "linf_over_tau": round(err / tau, 4)}
    if kernels:
        m.mgard_timing(True)
        for _ in range(2):
            m.mgard_compress(u, tol, out=out, **kw)
        torch.cuda.synchronize()
        rep = m.mgard_timing_report()
        m.mgard_timing(False)
        r["decompose_quantize_ms"] = round(sum(v[1] for k, v in rep.items() if k.startswith(
            ("coeff", "mass_restrict", "thomas", "add_", "maxabs", "r0_thomas0", "tail_decompose"))) / 2, 4)
    return r


def bench_workloads(m, torch, u513, steps=5):
    """The other workloads of the benchmark configuration: the 513^3 field at rel tol 1e-2 and
    1e-4, and the 500^3 float64 field on the geometric grid (ratio 1.01 per dimension, spectral
    k^-3 plus a tanh front, seed 3) at rel tol 1e-4, each timed as a round trip."""
    import fieldgen

    out = {}
    for tol in (1e-2, 1e-4):
        out[f"513^3 float32 k^-5/3, rel Linf {tol:g}"] = timed_round_trip(m, torch, u513, tol, steps)
        print(f"[bench] 513^3 tol {tol:g} done", file=sys.stderr, flush=True)
    print("[bench] generating 500^3 float64 geometric-grid field", file=sys.stderr, flush=True)
    u, coords = fieldgen.front3d(500, 3, 1.01, device="cuda")
    u = u.to(torch.float64).contiguous()
    m.mgard_autotune(u, coords)
    r = timed_round_trip(m, torch, u, 1e-4, steps, coords=coords, kernels=True)
    N = u.numel()
    sizes = [500]
    while sizes[-1] > 3:
        sizes.append(sizes[-1] // 2 + 1)
    # read u once, write 2-byte symbols, the coarse grids' round trips
    alg = N * 8 + 2 * N + 2 * 8 * sum(x ** 3 for x in sizes[1:])
    r["decompose_quantize_alg_GBps"] = round(alg / (r["decompose_quantize_ms"] * 1e-3) / 1e9, 1)
    r["decompose_quantize_frac"] = round(r["decompose_quantize_alg_GBps"] / HBM_PEAK_GBS, 4)
    out["500^3 float64 geometric grid, k^-3 + tanh front, rel Linf 1e-4"] = r
    print("[bench] 500^3 float64 done", file=sys.stderr, flush=True)
    del u
    torch.cuda.empty_cache()
    return out


def bench_refactor(m, torch, u, tol=1e-3, reps=3):
    """Refactoring of the 513^3 field into 32 bitplanes per level, the retrieval plan for rel
    L-inf tol, reconstruction from the planned segments; fetched bytes raw and after the
    second lossless stage."""
    buf, nb = m.mgard_refactor(u, 32)
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(reps):
        m.mgard_refactor(u, 32, out=buf)
    torch.cuda.synchronize()
    t_ref = (time.perf_counter() - a) / reps
    head = buf[:1 << 16].cpu().numpy().tobytes()
    mb, L, B, tot = m.mgard_refactor_inspect(head)
    head = head[:mb]
    want, est = m.mgard_refactor_request(head, tol)
    rec = m.mgard_reconstruct(buf, nb, want)
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(reps):
        m.mgard_reconstruct(buf, nb, want, out=rec)
    torch.cuda.synchronize()
    t_rec = (time.perf_counter() - a) / reps
    err = float((rec.double() - u.double()).abs().max())
    tau = tol * float(u.abs().max())
    assert err <= tau, f"refactoring: L-infinity error {err} exceeds {tau}"
    ranges = m.mgard_refactor_ranges(head, None, want)
    fetched = sum(n for _, n in ranges)
    coded = 0
    for off, n in ranges:
        _, cb = m.mgard_lossless_encode(buf[off:off + n], n)
        coded += cb
    in_bytes = u.numel() * 4
    print(f"[bench] refactor: {t_ref * 1e3:.1f} ms, reconstruct {t_rec * 1e3:.1f} ms", file=sys.stderr, flush=True)
    return {"workload": f"513^3 float32 k^-5/3 (seed 2), 32 bitplanes per level, request rel Linf {tol:g}",
            "refactored_bytes": nb, "refactor_ms": round(t_ref * 1e3, 3), "refactor_GBps": round(in_bytes / t_ref / 1e9, 3),
            "planes": want, "fetched_bytes": fetched, "fetched_bytes_lossless": coded,
            "reconstruct_ms": round(t_rec * 1e3, 3), "reconstruct_GBps": round(in_bytes / t_rec / 1e9, 3),
            "linf_over_tau": round(err / tau, 4), "estimate_over_tau": round(est / tau, 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=513)
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--chunk", type=int, default=1024, help="symbols per Huffman chunk (a multiple of 256)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=145)
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-field batch measurement")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-allocation ratio")
    ap.add_argument("--no-chunked", action="store_true", help="skip the out-of-core (host-resident) measurement")
    ap.add_argument("--only-batch", action="store_true", help="run only the 256-field batch measurement")
    ap.add_argument("--no-tune", action="store_true", help="use the default launch shapes")
    ap.add_argument("--no-workloads", action="store_true", help="skip the other tolerances and the float64 field")
    ap.add_argument("--no-refactor", action="store_true", help="skip the refactoring measurement")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of this many MiB three times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; the path has no multi-GPU mode "
                                   "(fields shard by independent chunks, see the design notes)"}))
        sys.exit(2)

    import numpy as np
    import torch

    import fieldgen
    import paper_2401_05994_amd as m

    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.only_batch:
        print(json.dumps({"batched": bench_batch(m, torch)}))
        return
    if args.calib_copy > 0:
        src = torch.ones(args.calib_copy << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)  # elementwise: reads and writes calib_copy MiB
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: 3 x {args.calib_copy} MiB", file=sys.stderr, flush=True)
        del src, dst
    n = args.n
    print(f"[bench] generating {n}^3 float32 field", file=sys.stderr, flush=True)
    u = fieldgen.spectral((n, n, n), -5.0 / 3.0, 2, device=dev).to(torch.float32).contiguous()
    in_bytes = u.numel() * 4
    bound = m.mgard_compress_bound(u.shape, m.F32, chunk=args.chunk)
    out = torch.empty(bound, dtype=torch.uint8, device=dev)
    rec = torch.empty_like(u)

    def step():
        buf, nb, info = m.mgard_compress(u, args.tol, chunk=args.chunk, out=out)
        m.mgard_decompress(buf, nb, out=rec)
        return nb, info

    tuned = not args.no_tune
    if tuned:
        # the library's launch-shape tuner, once per level shape, before anything is timed
        t_tune = time.perf_counter()
        m.mgard_autotune(u)
        print(f"[bench] autotuned in {time.perf_counter() - t_tune:.1f} s", file=sys.stderr, flush=True)

    for i in range(args.warmup):
        step()
        print(f"[bench] warmup {i + 1}/{args.warmup}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tc = td = 0.0
    t0 = time.perf_counter()
    for i in range(args.steps):
        a = time.perf_counter()
        buf, nb, info = m.mgard_compress(u, args.tol, chunk=args.chunk, out=out)
        b = time.perf_counter()
        m.mgard_decompress(buf, nb, out=rec)
        torch.cuda.synchronize()
        c = time.perf_counter()
        tc += b - a
        td += c - b
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) / args.steps * 1e3
    print(f"[bench] timed {args.steps} steps: {ms:.2f} ms/step", file=sys.stderr, flush=True)
    err = float((rec - u).abs().max())
    tau = info["tau_abs"]
    assert err <= tau, f"L-infinity error {err} exceeds the bound {tau}"

    # kernel durations with HIP events on the launch stream (separate pass)
    m.mgard_timing(True)
    kt_steps = 2
    for _ in range(kt_steps):
        step()
    torch.cuda.synchronize()
    rep = m.mgard_timing_report()
    m.mgard_timing(False)
    comp_kernels = {k: v for k, v in rep.items()}
    dom = max(comp_kernels, key=lambda k: comp_kernels[k][1])
    sizes = []
    s = n
    while s > 3:
        sizes.append(s)
        s = s // 2 + 1
    sizes.append(3)
    sizes = sizes[::-1]
    roof_kernel = "coeff_r21_fine"
    launches, total_ms = rep[roof_kernel]
    avg_ms = total_ms / launches
    alg = algorithmic_bytes(roof_kernel, n, 4, sizes)
    inter = sizes[-1] * sizes[-2] * sizes[-2] * 4  # the plane restricted along dims 2 and 1
    achieved = alg / (avg_ms * 1e-3) / 1e9
    decomp_ms = sum(v[1] for k, v in rep.items()
                    if k.startswith(("coeff", "mass_restrict", "thomas", "add_", "maxabs", "r0_thomas0")) and "sub" not in k) / kt_steps
    N = u.numel()
    alg_dq = N * 4 + 2 * N + 2 * 4 * sum(x ** 3 for x in sizes[:-1])  # read u, write symbols, coarse grids

    result = {
        "metric": "compress+decompress GB/s at rel Linf 1e-3 (% HBM peak); ratio learned vs plain",
        "value": round(in_bytes / (ms * 1e-3) / 1e9, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"3D {n}^3 float32 spectral k^-5/3 field (seed 2), rel Linf tol {args.tol}, "
                               "compress+decompress round trip, plain allocation",
                   "tol": args.tol, "shape": [n, n, n], "autotuned": tuned},
        "compress_GBps": round(in_bytes * args.steps / tc / 1e9, 3),
        "decompress_GBps": round(in_bytes * args.steps / td / 1e9, 3),
        "ratio": round(in_bytes / nb, 4),
        "linf_over_tau": round(err / tau, 4),
        "roofline": {"bound": "hbm", "kernel": roof_kernel, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(n, args.tol), "avg_ms": round(avg_ms, 4), "alg_bytes": alg,
                     "intermediate_bytes": inter,
                     "frac_with_intermediate": round((alg + inter) / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "dominant_kernel": {"name": dom, "ms_per_step": round(rep[dom][1] / kt_steps, 4)},
        "decompose_quantize": {"ms": round(decomp_ms, 4),
                               "alg_GBps": round(alg_dq / (decomp_ms * 1e-3) / 1e9, 1),
                               "frac": round(alg_dq / (decomp_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "kernels_ms_per_step": {k: round(v[1] / kt_steps, 4) for k, v in sorted(rep.items())},
    }

    # the learned allocation on the same field and tolerance (outside the timed region)
    from paper_2401_05994_amd import learned as lrn

    if not args.no_learned and os.path.exists(lrn.DEFAULT_MODEL):
        params, _ = lrn.load()
        model = m.Model(params)
        torch.cuda.synchronize()
        a = time.perf_counter()
        lbuf, lnb, linfo = m.mgard_compress_learned(u, args.tol, model, out=out)
        torch.cuda.synchronize()
        lms = (time.perf_counter() - a) * 1e3
        lrec = m.mgard_decompress(lbuf, lnb, out=rec)
        lerr = float((lrec - u).abs().max())
        assert lerr <= linfo["tau_abs"], f"learned: L-infinity error {lerr} exceeds {linfo['tau_abs']}"
        result["learned"] = {"ratio_learned": round(in_bytes / lnb, 4), "ratio_plain": round(in_bytes / nb, 4),
                             "learned_over_plain": round(nb / lnb, 4), "fallback": int(linfo["fallback_used"]),
                             "linf_over_tau": round(lerr / linfo["tau_abs"], 4), "compress_ms": round(lms, 2)}
        print(f"[bench] learned: ratio {in_bytes / lnb:.3f} vs plain {in_bytes / nb:.3f}", file=sys.stderr,
              flush=True)

    # the lossless stage on the same stream (outside the timed region)
    lbuf, lnb, _ = m.mgard_compress(u, args.tol, chunk=args.chunk, lossless=True)
    result["lossless_stage"] = {"ratio_without": round(in_bytes / nb, 4), "ratio_with": round(in_bytes / lnb, 4)}
    del lbuf

    if not args.no_workloads:
        result["workloads"] = bench_workloads(m, torch, u)

    if not args.no_refactor:
        result["refactor"] = bench_refactor(m, torch, u)

    if not args.no_batch:
        result["batched"] = bench_batch(m, torch)

    if not args.no_chunked:
        result["chunked"] = bench_chunked(m, torch)

    if not args.no_cpu_baseline:
        from oracle import codec

        cn = args.cpu_n
        cu = fieldgen.spectral((cn, cn, cn), -5.0 / 3.0, 2).astype(np.float32)
        print(f"[bench] cpu oracle on {cn}^3", file=sys.stderr, flush=True)
        from threadpoolctl import threadpool_limits

        with threadpool_limits(limits=1):
            a = time.perf_counter()
            cb = codec.compress(cu, args.tol)
            codec.decompress(cb)
            dt = time.perf_counter() - a
        # the same sample with the host's BLAS / FFT thread pools unrestricted: the oracle's
        # numpy steps may then use several threads, its pure-Python Huffman one
        a = time.perf_counter()
        cb = codec.compress(cu, args.tol)
        codec.decompress(cb)
        dt_all = time.perf_counter() - a
        ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        model = ""
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
        result["cpu_baseline"] = {
            "value": round(cu.nbytes / dt / 1e9, 6), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"{cn}^3 float32 field of the same generator and tolerance, compress+decompress "
                      f"round trip ({dt:.1f} s, numpy + pure-Python Huffman, one thread)",
            "cpu_model": model, "host_cpus": ncpu,
            "all_threads": {"value": round(cu.nbytes / dt_all / 1e9, 6), "threads_available": ncpu,
                            "seconds": round(dt_all, 2)},
        }
    print(json.dumps(result))


if __name__ == "__main__":
    main()
