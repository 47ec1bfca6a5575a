"""Throughput benchmark of the batched FP32 multichannel-interpolation workload on one GPU.

Workload (default): 65536 independent real signals, each observed through M = 3
derivative channels {f, f', f''} with N = 1366 samples per channel (band of
mu = 4098 coefficients, [-2048, 2049]), reconstructed on a 16384-point grid (4x the
4096-sample signal length), FP32 transforms.  Inputs are seeded synthetic signals with
spectrum e^{-0.01|n|} CN(0,1) + 1e-3 CN(0,1) out to |n| = 8192 (not bandlimited): a
pool of 8192 distinct signals tiled 8 times, resident in HBM before timing starts.

A step is one mci_reconstruct_1d call over the whole batch (every step of the method:
channel DFTs, per-residue apply, placement on the output grid, inverse DFT).  Prints
one JSON line with throughput (reconstructed output samples/s), the roofline of the
dominant kernel (timed with HIP events on its stream) and the FP64 CPU oracle on a
bounded sample of the same workload, plus the relative error of that sample.  The
default line also carries the metric's 2-D part under "sisr2" and "sisr4": 256
grayscale images upsampled x2 (256^2 -> 512^2) and x4 (128^2 -> 512^2), each with its
own time, output px/s, roofline, oracle baseline, errors and PSNR (--no-2d skips them),
and, outside the metric, the uneven batch under "uneven" (4096 mixed 1-D and 2-D instances
in one graph launch, with its oracle check; --no-uneven skips it) and the refiner's forward
throughput under "refiner_forward" (initial weights; --no-refiner skips it).

  python bench.py [--steps K] [--warmup W] [--workload batched1d|sisr2|sisr4|sisr3|refiner|uneven|offgrid|errsel]
                  [--no-cpu]
                  [--storage f32|f16] [--lanes 16]
"""
import argparse
import copy
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
FP32_VALU_PEAK_TFLOPS = 157.3   # vendor figure (packed FP32); 78.6 without packed instructions
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz: the FP32 vector peak without packed
# FP32 instructions, which this build does not emit
FP32_VALU_UNPACKED_TFLOPS = 78.6


def mci1d_flops(M, N, n_out):
    """Algorithmic flops of one real-mode 1-D reconstruction: M real-input DFTs of length N
    (2.5 N log2 N each), the per-coefficient M-term apply (8 flops per complex multiply-add
    over the M N band coefficients), and one real-output inverse DFT of length n_out."""
    import math
    return M * 2.5 * N * math.log2(N) + 8.0 * M * (M * N) + 2.5 * n_out * math.log2(n_out)
METRIC = "reconstructed samples/s (1-D batch, 2-D ×2/×4) vs HBM roofline; rel err vs FP64"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="batched1d",
                    choices=["batched1d", "sisr2", "sisr4", "sisr3", "refiner", "uneven", "offgrid", "errsel"])
    ap.add_argument("--storage", default="f32", choices=["f32", "f16"], help="uneven: storage of the packed buffers")
    ap.add_argument("--lanes", type=int, default=16, help="uneven: concurrent lanes of the batch")
    ap.add_argument("--pairs", type=int, default=20000, help="refiner: training pairs")
    ap.add_argument("--epochs", type=int, default=3, help="refiner: training epochs")
    ap.add_argument("--batch", type=int, default=0, help="override the batch size (0 = workload default)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/mci1d_batched_fp32_traffic.json from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--no-2d", action="store_true",
                    help="batched1d: skip the 2-D x2 and x4 workloads that the default line also carries")
    ap.add_argument("--no-uneven", action="store_true",
                    help="batched1d: skip the uneven-batch workload that the default line also carries")
    ap.add_argument("--no-refiner", action="store_true",
                    help="batched1d: skip the refiner forward throughput that the default line also carries")
    ap.add_argument("--cpu-sample", type=int, default=0, help="signals/images in the CPU sample (0 = default)")
    return ap.parse_args()


def source_hash(paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


FUSED_SOURCES = ["paper_1802_10291_amd/csrc/mci_fused.hip", "paper_1802_10291_amd/csrc/mci_device.h"]
FUSED_KERNEL = "void mci::k_mci1d_fused<1024, 2, 4096, 4, 3, 1, float>(mci::FusedArgs)"


def write_traffic(fetch_dir, write_dir, units=65536):
    """HBM traffic of the batched workload's fused kernel from two rocprofv3 --pmc runs of this
    script (FETCH_SIZE, then WRITE_SIZE; counter_collection.csv in each directory), each scaled
    by what the counter reads for the 2 GiB device-to-device copy of copy_bandwidth() in the same
    run; written to profiles/ with the hash of the kernel's source.  No GPU is used."""
    import csv
    import glob

    def per_kernel(d, counter):
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        fused, copy = [], []
        for f in files:
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] != counter:
                    continue
                v = float(r["Counter_Value"]) * 1024.0          # KiB per dispatch
                if "k_mci1d_fused" in r["Kernel_Name"]:
                    fused.append(v)
                elif "copyBuffer" in r["Kernel_Name"]:               # the runtime's device-to-device copy
                    copy.append((int(r["Grid_Size"]), v))
        big = max(g for g, _ in copy)                            # the 2 GiB copy has the largest grid
        return float(np.mean(fused)), float(np.median([v for g, v in copy if g == big]))

    nbytes = 2 << 30
    f_fused, f_copy = per_kernel(fetch_dir, "FETCH_SIZE")
    w_fused, w_copy = per_kernel(write_dir, "WRITE_SIZE")
    fc, wc = nbytes / f_copy, nbytes / w_copy
    doc = {"kernel": FUSED_KERNEL, "units_per_launch": units, "hbm_bytes_per_launch": f_fused * fc + w_fused * wc,
           "read_bytes": f_fused * fc, "write_bytes": w_fused * wc, "fetch_calibration": fc, "write_calibration": wc,
           "kernel_source_hash": source_hash(FUSED_SOURCES)}
    with open(os.path.join(ROOT, "profiles", "mci1d_batched_fp32_traffic.json"), "w") as fh:
        json.dump(doc, fh, indent=1)
    print(json.dumps(doc))


def load_traffic(name, khash, per_launch_units):
    """HBM traffic per launch from the committed rocprofv3 counter summary, if it was
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"{name}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_hash") != khash or t.get("units_per_launch") != per_launch_units:
        return None
    return t.get("hbm_bytes_per_launch")


def rel_errors(got, want, unit_name, count=None):
    """Per result (the leading axis): relative L2 ||y - y_ref|| / ||y_ref|| and the element-wise
    error max |y - y_ref| / max |y_ref|; reported as max and median of each."""
    n = got.shape[0]
    d = (got - want).reshape(n, -1)
    w = want.reshape(n, -1)
    l2 = np.linalg.norm(d, axis=1) / np.maximum(np.linalg.norm(w, axis=1), 1e-300)
    mx = np.abs(d).max(axis=1) / np.maximum(np.abs(w).max(axis=1), 1e-300)
    return {"max": float(l2.max()), "median": float(np.median(l2)),
            "max_abs_over_ref_inf_max": float(mx.max()), "max_abs_over_ref_inf_median": float(np.median(mx)),
            unit_name: int(count if count is not None else n)}


def time_steps(torch, fn, steps, warmup, stream):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [a.elapsed_time(b) for a, b in evs]
    return wall, per


def copy_bandwidth(torch, nbytes=2 << 30):
    """Achievable HBM bandwidth of a plain device-to-device copy (read + write bytes)."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(10):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / 10
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9


def bench_batched1d(args, torch):
    from paper_1802_10291_amd import Plan1D
    from synth import signals as S

    B = args.batch or 65536
    M, N, n_out, n_max = 3, 1366, 16384, 8192
    pool = min(8192, B)
    log(f"generating {pool} seeded signals (tiled to {B})")
    from concurrent.futures import ThreadPoolExecutor
    host = np.empty((pool, M, N), dtype=np.float32)
    chunk = 256

    def work(c):
        n = min(chunk, pool - c)
        host[c:c + n] = S.smooth_noisy_batch(c, n, M, N, n_max)

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(work, range(0, pool, chunk)))
    dev_pool = torch.from_numpy(host).cuda()
    g = dev_pool.repeat((B + pool - 1) // pool, 1, 1)[:B].contiguous()
    del dev_pool
    plan = Plan1D(N=N, n_out=n_out, channels=[("deriv", 0), ("deriv", 1), ("deriv", 2)], precision="f32")
    info = plan.info
    y = torch.empty((B, 1, n_out), dtype=torch.float32, device="cuda")
    ws, need = plan.workspace(B)
    stream = torch.cuda.current_stream()
    log(f"plan: path={'fused' if info.path else 'multi-pass'} fwd_len={info.fft_len_fwd} inv_len={info.fft_len_inv} "
        f"max_cond={info.max_cond:.3g} workspace={need / 2**30:.2f} GiB")

    def step():
        plan.reconstruct(g, out=y)

    wall, per = time_steps(torch, step, args.steps, args.warmup, stream)
    ms = float(np.mean(per))
    samples = B * n_out
    value = samples * args.steps / (sum(per) * 1e-3)
    alg_bytes = B * (M * N * 4 + n_out * 4)
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    kernel_src = FUSED_SOURCES if info.path \
        else ["paper_1802_10291_amd/csrc/mci_kernels.hip", "paper_1802_10291_amd/csrc/mci_device.h"]
    khash = source_hash(kernel_src)
    traffic = load_traffic("mci1d_batched_fp32", khash, B) if info.path else None
    result = {
        "metric": METRIC, "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "1-D batched FP32 MCI: 65536 signals x M=3 derivative channels {f,f',f''} x N=1366 "
                               "samples (band mu=4098, [-2048,2049]) -> 16384-point grid",
                   "batch": B, "M": M, "N": N, "n_out": n_out, "path": "fused" if info.path else "multi-pass"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "mci1d fused" if info.path else "whole multi-pass step",
                     "algorithmic_bytes_per_launch": alg_bytes, "kernel_source_hash": khash},
        "alu_algorithmic": {"achieved": B * mci1d_flops(M, N, n_out) / (ms * 1e-3) / 1e12,
                            "peak": FP32_VALU_UNPACKED_TFLOPS, "unit": "TFLOP/s",
                            "frac": B * mci1d_flops(M, N, n_out) / (ms * 1e-3) / 1e12 / FP32_VALU_UNPACKED_TFLOPS,
                            "flops_per_signal": mci1d_flops(M, N, n_out)},
        "wall_s": wall,
    }
    # CPU oracle on a bounded sample of the same workload
    if not args.no_cpu:
        from oracle import oracle as O
        ns = args.cpu_sample or 512
        idx = np.linspace(0, B - 1, ns).astype(np.int64)
        g_s = g[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.float64)
        y_s = y[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.float64)
        ch = O.Channels(N=N, kinds=[O.MULT_DERIV] * 3, orders=[0, 1, 2])
        log(f"CPU oracle on {ns} signals with {O.num_threads()} threads")
        t0 = time.perf_counter()
        want = O.reconstruct_1d(ch, g_s, n_out)
        dt = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": ns * n_out / dt, "unit": "samples/s", "cores": O.num_threads(),
                                  "kind": "oracle",
                                  "sample": f"{ns} of the {B} signals (evenly spaced indices), FP64 direct DFT + "
                                            f"Gaussian elimination + direct trigonometric sum; {dt:.1f} s"}
        result["rel_err_vs_fp64_oracle"] = rel_errors(y_s, want, "signals")
    result["copy_bandwidth_GBs"] = copy_bandwidth(torch)
    return result


def bench_offgrid(args, torch):
    """Off-grid evaluation: the batched workload's signals ({f, f', f''}, N = 1366, band 4098)
    evaluated at 16384 seeded uniform random points in [0, 2 pi) shared by the batch."""
    from paper_1802_10291_amd import OffGrid, _lib
    from synth import signals as S

    B = args.batch or 16384
    M, N, n_max, n_t = 3, 1366, 8192, 16384
    pool = min(2048, B)
    log(f"generating {pool} seeded signals (tiled to {B})")
    from concurrent.futures import ThreadPoolExecutor
    host = np.empty((pool, M, N), dtype=np.float32)

    def work(c):
        n = min(256, pool - c)
        host[c:c + n] = S.smooth_noisy_batch(c, n, M, N, n_max)

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(work, range(0, pool, 256)))
    g = torch.from_numpy(host).cuda().repeat((B + pool - 1) // pool, 1, 1)[:B].contiguous()
    t_host = np.random.default_rng(2024).uniform(0.0, 2 * np.pi, size=n_t)
    t = torch.from_numpy(t_host).cuda()
    og = OffGrid(N=N, channels=[("deriv", 0), ("deriv", 1), ("deriv", 2)], precision="f32")
    y = torch.empty((B, 1, n_t), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    L, w = og.grid_len, og.width
    log(f"grid length {L}, kernel width {w}")

    def step():
        og.evaluate(g, t, out=y)

    wall, per = time_steps(torch, step, args.steps, args.warmup, stream)
    ms = float(np.mean(per))
    # the grid stage alone (the grid plan of the same off-grid plan, same input)
    gp = _lib.mci_offgrid_info(og.handle)[3]
    gneed = _lib.mci_workspace_size(gp, B)
    gws = torch.empty(max(gneed, 1), dtype=torch.uint8, device="cuda")
    gy = torch.empty((B, 1, L), dtype=torch.float32, device="cuda")
    sh = int(stream.cuda_stream)

    def grid_step():
        _lib.mci_reconstruct_1d(gp, g.data_ptr(), gy.data_ptr(), B, gws.data_ptr(), gneed, sh)

    _, gper = time_steps(torch, grid_step, args.steps, args.warmup, stream)
    del gy, gws
    ms_grid = float(np.mean(gper))
    value = B * n_t * args.steps / (sum(per) * 1e-3)
    alg_bytes = B * (M * N * 4 + n_t * 4) + n_t * 8
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    result = {
        "metric": METRIC, "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"1-D off-grid FP32 MCI: {B} signals x M=3 derivative channels {{f,f',f''}} x N=1366 "
                               f"samples (band mu=4098) evaluated at {n_t} random points shared by the batch "
                               f"(grid {L}, kernel width {w})",
                   "batch": B, "M": M, "N": N, "n_t": n_t, "grid_len": L, "width": w},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "whole off-grid step",
                     "algorithmic_bytes_per_launch": alg_bytes},
        "stages_ms": {"grid": ms_grid, "gather": ms - ms_grid},
        # the gather stage on its own: it reads the grid once and writes the outputs
        "gather_roofline": {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
                            "algorithmic_bytes": B * (L + n_t) * 4,
                            "achieved": B * (L + n_t) * 4 / ((ms - ms_grid) * 1e-3) / 1e9,
                            "frac": B * (L + n_t) * 4 / ((ms - ms_grid) * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "wall_s": wall,
    }
    if not args.no_cpu:
        from oracle import oracle as O
        ch = O.Channels(N=N, kinds=[O.MULT_DERIV] * 3, orders=[0, 1, 2])
        idx = np.linspace(0, B - 1, 64).astype(np.int64)
        g_s = g[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.float64)
        y_s = y[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.float64)
        log(f"CPU oracle: direct sums at {n_t} points per signal, up to 64 signals or ~15 s")
        t0 = time.perf_counter()
        wants = []
        for k in range(len(idx)):
            a = O.recover_band(ch, g_s[k])
            wants.append(O.evaluate_band(a, ch.n1, t_host))
            if time.perf_counter() - t0 > 15.0:
                break
        dt = time.perf_counter() - t0
        ns = len(wants)
        result["cpu_baseline"] = {"value": ns * n_t / dt, "unit": "samples/s", "cores": 1, "kind": "oracle",
                                  "sample": f"{ns} of the {B} signals (evenly spaced indices), FP64 direct DFT + "
                                            f"Gaussian elimination + direct sum at each of the {n_t} points; "
                                            f"{dt:.1f} s"}
        result["rel_err_vs_fp64_oracle"] = rel_errors(y_s[:ns, 0], np.stack(wants), "signals")
    return result


ERR_CANDIDATES = [  # (N, channels, n1 shift from the default): about 4098 samples each
    (4098, [("deriv", 0)], 0), (2049, [("deriv", 0), ("deriv", 1)], 0),
    (1366, [("deriv", 0), ("deriv", 1), ("deriv", 2)], 0), (2049, [("deriv", 0), ("hilbert", 0)], 0),
    (1025, [("deriv", 0), ("deriv", 1), ("deriv", 2), ("deriv", 3)], 0),
    (2049, [("deriv", 0), ("deriv", 1)], 64), (4098, [("deriv", 0)], -64),
    (1366, [("deriv", 0), ("deriv", 1), ("deriv", 2)], 32)]


def bench_errsel(args, torch):
    """Averaged-error scoring (Theorem 4.4): 16384 signals with coefficients on |n| <= 8192
    against 8 candidate plans of about 4098 samples, and the plan of least error per signal."""
    from paper_1802_10291_amd import Plan1D, _lib
    from synth import signals as S
    from oracle import oracle as O

    B = args.batch or 16384
    n_max = 8192
    n_lo, n_span = -n_max, 2 * n_max + 1
    pool = min(512, B)
    log(f"generating {pool} seeded spectra (tiled to {B})")
    rng = np.random.default_rng(31)
    host = np.empty((pool, n_span), dtype=np.complex64)
    for k in range(pool):
        host[k] = S.smooth_noisy_spectrum(rng, n_max)[1]
    a = torch.from_numpy(host).cuda().repeat((B + pool - 1) // pool, 1)[:B].contiguous()
    plans, chans = [], []
    for N, channels, shift in ERR_CANDIDATES:
        mu = N * len(channels)
        n1 = O.default_n1(mu) + shift
        plans.append(Plan1D(N=N, n_out=2 * mu, channels=channels, n1=n1))
        chans.append(O.Channels(N=N, kinds=[O.MULT_HILBERT if k == "hilbert" else O.MULT_DERIV for k, _ in channels],
                                orders=[int(v) for _, v in channels], n1=n1))
    C = len(plans)
    eps = torch.empty((B, C), dtype=torch.float64, device="cuda")
    best = torch.empty((B,), dtype=torch.int32, device="cuda")
    need = _lib.mci_averaged_error_workspace_size(C, n_span, _lib.MCI_F32)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    handles = [p.handle for p in plans]

    def step():
        _lib.mci_averaged_error(handles, a.data_ptr(), n_lo, n_span, B, _lib.MCI_F32, eps.data_ptr(), best.data_ptr(),
                                ws.data_ptr(), need, sh)

    wall, per = time_steps(torch, step, args.steps, args.warmup, stream)
    ms = float(np.mean(per))
    alg_bytes = B * n_span * 8 + B * (C * 8 + 4)
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    counts = np.bincount(best.cpu().numpy(), minlength=C)
    result = {
        "metric": METRIC, "value": B * args.steps / (sum(per) * 1e-3), "unit": "signals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"averaged-error scoring (Theorem 4.4): {B} signals with coefficients on |n| <= {n_max} "
                               f"against {C} candidate plans of ~4098 samples (M = 1..4, derivative / Hilbert channels, "
                               "shifted bands), least-error plan per signal",
                   "batch": B, "n_span": n_span, "plans": C},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "weights + scoring pass",
                     "algorithmic_bytes_per_launch": alg_bytes},
        "chosen_plan_counts": counts.tolist(),
        "wall_s": wall,
    }
    if not args.no_cpu:
        n = np.arange(n_lo, n_lo + n_span)
        e_h = eps.cpu().numpy()
        log("CPU oracle: eq. averageerror per (signal, plan), up to ~15 s")
        t0 = time.perf_counter()
        errs, done = [], 0
        for k in range(0, B, max(1, B // 4096)):
            ref = host[k % pool].astype(np.complex128)
            want = np.array([O.averaged_error(ch, n, ref) for ch in chans])
            errs.append(float(np.max(np.abs(e_h[k] - want) / want)))
            done += 1
            if time.perf_counter() - t0 > 15.0:
                break
        dt = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": done / dt, "unit": "signals/s", "cores": 1, "kind": "oracle",
                                  "sample": f"{done} of the {B} signals (evenly spaced), each against the {C} plans: "
                                            f"FP64 inverse tables + eq. averageerror term by term; {dt:.1f} s"}
        result["rel_err_vs_fp64_oracle"] = {"max": float(np.max(errs)), "signals": done}
    return result


def bench_sisr(args, torch, s, M=2, HR=512):
    from paper_1802_10291_amd import Plan2D
    from synth import images as SI

    B = args.batch or 256
    H = W = HR
    h, w = H // s, W // s
    pool = min(32, B)
    log(f"generating {pool} seeded {H}x{W} images (tiled to {B}), decimating by {s}")
    hr_host = SI.random_field_images(0, pool, H, W)
    lr_host = SI.decimate(hr_host, s)
    lr = torch.from_numpy(lr_host).cuda().repeat((B + pool - 1) // pool, 1, 1)[:B].contiguous()
    plan = Plan2D(h, w, s, channels=M)
    out = torch.empty((B, H, W), dtype=torch.float32, device="cuda")
    ws, need = plan.workspace(B)
    stream = torch.cuda.current_stream()

    def step():
        plan.upsample(lr, out=out)

    wall, per = time_steps(torch, step, args.steps, args.warmup, stream)
    ms = float(np.mean(per))
    px = B * H * W
    value = px * args.steps / (sum(per) * 1e-3)
    alg_bytes = B * (h * w * 4 + H * W * 4)
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    # quality vs the ground-truth images
    up = out[:pool].cpu().numpy().astype(np.float64)
    from oracle import oracle as O
    psnr = [O.psnr(up[i], hr_host[i].astype(np.float64)) for i in range(pool)]
    result = {
        "metric": METRIC, "value": value, "unit": "px/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"2-D separable MCI x{s}: {B} images {h}x{w} -> {H}x{W}, M={M} (line + centred "
                               "difference" + (" + second difference" if M == 3 else "") + ") per axis",
                   "batch": B, "scale": s, "channels": M, "path": "line pass" if plan.info.path else "multi-pass"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "whole 2-D step",
                     "algorithmic_bytes_per_launch": alg_bytes},
        "psnr_db_mean": float(np.mean(psnr)),
        "wall_s": wall,
    }
    if not args.no_cpu:
        # the oracle image by image over the distinct images, cycling through them until about
        # 10 s have passed (or --cpu-sample images); the first pass gives the errors
        ns_max = args.cpu_sample or 100000
        t0 = time.perf_counter()
        wants, done = [], 0
        while done < ns_max and (done < pool or time.perf_counter() - t0 < 10.0):
            yi = O.upsample_2d(lr_host[done % pool].astype(np.float64), s, M=M)
            if done < pool:
                wants.append(yi)
            done += 1
        dt = time.perf_counter() - t0
        ns = len(wants)
        want = np.stack(wants)
        result["cpu_baseline"] = {"value": done * H * W / dt, "unit": "px/s", "cores": O.num_threads(),
                                  "kind": "oracle",
                                  "sample": f"{done} image upsamples cycling over the {pool} distinct images "
                                            f"(until ~10 s); {dt:.1f} s"}
        result["rel_err_vs_fp64_oracle"] = rel_errors(up[:ns], want, "images")
    return result


def scaled_deriv_tables(M, N):
    """(i n / N)^m on the default band of M N coefficients."""
    mu = M * N
    n = np.arange(-((mu - 1) // 2), -((mu - 1) // 2) + mu)
    return [(1j * n / N) ** m for m in range(M)]


def bench_uneven(args, torch):
    """The mixed workload: 4096 instances (3584 1-D signals of 17 lengths x 3 channel counts,
    512 images of 9 sizes) in one uneven batch, captured as one graph."""
    from concurrent.futures import ThreadPoolExecutor
    from paper_1802_10291_amd import Batch, Plan1D, Plan2D
    from synth import uneven as U

    f16 = args.storage == "f16"
    np_dt = np.float16 if f16 else np.float32
    esz = 2 if f16 else 4
    storage = "f16" if f16 else "native"
    items = U.instances()
    cls = U.classes(items)
    keys = list(cls)
    log(f"{len(items)} instances in {len(keys)} size classes; storage {storage}")
    plans, pools = {}, {}
    pool_n = 4

    def make_pool(ci):
        k = keys[ci]
        pools[k] = U.class_pool(k, ci, min(pool_n, len(cls[k])), dtype=np_dt, scaled=f16)

    with ThreadPoolExecutor(max_workers=8) as ex:
        list(ex.map(make_pool, range(len(keys))))
    for k in keys:
        if k[0] == "1d":
            _, L, M = k
            N = -(-L // M)
            chans = [("table", t) for t in scaled_deriv_tables(M, N)] if f16 else [("deriv", m) for m in range(M)]
            plans[k] = Plan1D(N=N, n_out=4 * L, channels=chans, storage=storage)
        else:
            plans[k] = Plan2D(k[1] // 2, k[1] // 2, 2, storage=storage)
    # autotune every class at its own instance count (cache: $MCI_TUNE_CACHE if set)
    cache = os.environ.get("MCI_TUNE_CACHE") or os.path.join("/tmp", f"mci_tune_{os.getpid()}.json")
    t0 = time.perf_counter()
    tuned = {k: plans[k].autotune(len(cls[k]), cache) for k in keys}
    log(f"autotuned {len(keys)} classes in {time.perf_counter() - t0:.1f} s")
    batch = Batch([plans[it.key()] for it in items], lanes=args.lanes)
    packed = np.zeros(batch.in_elems, dtype=np_dt)
    pos = {i: j for k in keys for j, i in enumerate(cls[k])}    # instance -> position in its class
    for i, (it, off) in enumerate(zip(items, batch.in_offsets)):
        k = it.key()
        x = pools[k][pos[i] % len(pools[k])].ravel()             # the class's first instance is pool entry 0
        packed[off:off + x.size] = x
    dev_in = torch.from_numpy(packed).cuda()
    dev_out = torch.zeros(batch.out_elems, dtype=dev_in.dtype, device="cuda")
    stream = torch.cuda.current_stream()
    in_bytes = sum(plans[it.key()].instance_sizes()[0] for it in items) * esz
    out_elems = sum(plans[it.key()].instance_sizes()[1] for it in items)
    alg_bytes = in_bytes + out_elems * esz
    log(f"packed input {batch.in_elems * esz / 2**30:.2f} GiB, output {batch.out_elems * esz / 2**30:.2f} GiB, "
        f"workspace {batch.ws_bytes / 2**30:.2f} GiB")

    def eager():
        batch.run(dev_in, dev_out)

    # eager timing, then one graph holding the whole batch
    _, per_eager = time_steps(torch, eager, max(3, args.steps // 2), args.warmup, stream)
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        eager()
    stream.wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        eager()
    wall, per = time_steps(torch, graph.replay, args.steps, args.warmup, stream)
    ms = float(np.mean(per))
    value = out_elems * args.steps / (sum(per) * 1e-3)
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    host_out = dev_out.cpu().numpy()

    # per class: time alone (dense batch of its instance count), bytes, error vs the oracle
    from oracle import oracle as O
    rows = []
    first_out = {}
    for i, (it, off) in enumerate(zip(items, batch.out_offsets)):
        if it.key() not in first_out:
            first_out[it.key()] = (i, off)
    per_class_err = {}

    def class_err(k):
        _, off = first_out[k]
        x = pools[k][0].astype(np.float64)
        n_o = plans[k].instance_sizes()[1]
        got = host_out[off:off + n_o].astype(np.float64)
        if k[0] == "2d":
            want = O.upsample_2d(x[None], 2)[0].ravel()
            return k, rel_errors(got[None], want[None], "instances"), "full"
        _, L, M = k
        N = -(-L // M)
        if f16:
            ch = O.Channels(N=N, kinds=[O.MULT_TABLE] * M, orders=[0] * M, tables=np.stack(scaled_deriv_tables(M, N)))
        else:
            ch = O.Channels(N=N, kinds=[O.MULT_DERIV] * M, orders=list(range(M)))
        if L <= 4096:
            want = O.reconstruct_1d(ch, x[None], 4 * L)[0, 0]
            return k, rel_errors(got[None], want[None], "instances"), "full"
        band = O.recover_band(ch, x[None])[0]
        idx = np.random.default_rng(L + M).choice(4 * L, 32, replace=False)
        want = O.evaluate_band(band, ch.n1, 2 * np.pi * idx / (4 * L))
        return k, rel_errors(got[idx][None], want[None], "instances"), "32 sampled points"

    cpu = None
    if not args.no_cpu:
        # CPU baseline: the oracle in full on the first instance of each small class (these also
        # give the classes' errors), then on further pool entries of them, until about 10 s
        small = [k for k in keys if (k[0] == "1d" and k[1] <= 4096) or (k[0] == "2d" and k[1] <= 256)]
        t0 = time.perf_counter()
        for k in small:
            per_class_err[k] = class_err(k)[1:]
        n_s = sum(plans[k].instance_sizes()[1] for k in small)
        extra = 0
        rounds = 0
        while time.perf_counter() - t0 < 10.0 and rounds < 1000:
            rounds += 1
            for k in small:
                if time.perf_counter() - t0 >= 10.0:
                    break
                x = pools[k][rounds % len(pools[k])].astype(np.float64)
                if k[0] == "2d":
                    O.upsample_2d(x[None], 2)
                else:
                    _, L, M = k
                    N = -(-L // M)
                    tabs = np.stack(scaled_deriv_tables(M, N)) if f16 else None
                    ch = O.Channels(N=N, kinds=[O.MULT_TABLE if f16 else O.MULT_DERIV] * M,
                                    orders=[0] * M if f16 else list(range(M)), tables=tabs)
                    O.reconstruct_1d(ch, x[None], 4 * L)
                n_s += plans[k].instance_sizes()[1]
                extra += 1
        dt = time.perf_counter() - t0
        cpu = {"value": n_s / dt, "unit": "samples/s", "cores": O.num_threads(), "kind": "oracle",
               "sample": f"{len(small) + extra} instances of the {len(small)} classes with L <= 4096 or side <= 256 "
                         f"(cycling over their pool entries until ~10 s), every output; {dt:.1f} s"}
        log(f"oracle on the large classes (sampled 1-D points, full 2-D images)")
        with ThreadPoolExecutor(max_workers=4) as ex:
            for k, e, how in ex.map(class_err, [k for k in keys if k not in per_class_err]):
                per_class_err[k] = (e, how)
    for k in keys:
        p = plans[k]
        n = len(cls[k])
        ni, no = p.instance_sizes()
        x = torch.from_numpy(np.stack([pools[k][j % len(pools[k])] for j in range(n)])).cuda()
        fn = (lambda: p.reconstruct(x)) if k[0] == "1d" else (lambda: p.upsample(x))
        _, pc = time_steps(torch, fn, 5, 2, stream)
        t = float(np.median(pc))
        name = f"1d L={k[1]} M={k[2]}" if k[0] == "1d" else f"2d {k[1] // 2}->{k[1]}"
        row = {"class": name, "instances": n, "variant": tuned[k][0], "ms": round(t, 4),
               "GBps": round(n * (ni + no) * esz / (t * 1e-3) / 1e9, 1)}
        if k in per_class_err:
            e = per_class_err[k][0]
            row["rel_err"], row["max_abs_over_ref_inf"], row["check"] = e["max"], e["max_abs_over_ref_inf_max"], \
                per_class_err[k][1]
        rows.append(row)
    result = {
        "metric": METRIC, "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"uneven batch, {'FP16' if f16 else 'FP32'} storage: {len(items)} instances "
                               f"({sum(1 for i in items if i.kind == '1d')} 1-D with L in 256..65536, M in 2..4, "
                               f"n_out = 4L; {sum(1 for i in items if i.kind == '2d')} 2-D x2 with sides 64..1024) "
                               f"in one graph launch", "classes": len(keys), "lanes": args.lanes,
                   "storage": storage},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "whole uneven-batch graph",
                     "algorithmic_bytes_per_launch": alg_bytes},
        "eager_ms_per_step": float(np.mean(per_eager)),
        # null when the oracle was not run (--no-cpu)
        "max_rel_err": max((r["rel_err"] for r in rows if "rel_err" in r), default=None),
        "max_abs_over_ref_inf": max((r["max_abs_over_ref_inf"] for r in rows if "rel_err" in r), default=None),
        "classes": rows,
        "wall_s": wall,
    }
    if cpu:
        result["cpu_baseline"] = cpu
    return result


def bench_refiner(args, torch, train=True):
    """Refiner workload: train on method-generated pairs, then time MCI alone and MCI + CNN on
    RGB 512 x 512 images upsampled x2 from 256 x 256, and report the PSNR gain.  train=False:
    the throughput only, on the initial weights (the kernels and their work do not depend on
    the weights' values), without training, PSNR or fallback."""
    from paper_1802_10291_amd import Plan2D, Refiner, upsample_rgb
    from paper_1802_10291_amd import refiner_train as RT

    r = Refiner(seed=0)
    hist, tau, t_train = [], None, 0.0
    p_mci = p_ref = frac = None
    n_eval = 512
    if train:
        t_train = time.perf_counter()
        hist, tau = RT.train(r, n_pairs=args.pairs, batch=16, size=512, lr=1e-3, epochs=args.epochs, log=log)
        t_train = time.perf_counter() - t_train
        p_mci, p_ref, frac = RT.evaluate(r, n_images=n_eval, size=512)
        log(f"held-out PSNR over {n_eval} images: MCI {p_mci:.3f} dB, MCI + CNN {p_ref:.3f} dB, refined {frac:.2f}")
    B = args.batch or 64
    hr_dev = RT.gpu_rgb_images([7_000_000 + i for i in range(min(B, 16))], 512)
    hr_dev = hr_dev.repeat((B + hr_dev.shape[0] - 1) // hr_dev.shape[0], 1, 1, 1)[:B].contiguous()
    lr_img = hr_dev[:, :, ::2, ::2].contiguous()
    plan = Plan2D(256, 256, 2)
    u = torch.empty_like(hr_dev)
    y = torch.empty_like(hr_dev)
    stream = torch.cuda.current_stream()
    w_mci, per_mci = time_steps(torch, lambda: upsample_rgb(plan, lr_img, out=u), args.steps, args.warmup, stream)
    ms_mci = float(np.mean(per_mci))

    def step():
        upsample_rgb(plan, lr_img, out=u)
        r.forward(u, fallback=train, out=y)

    wall, per = time_steps(torch, step, args.steps, args.warmup, stream)
    ms = float(np.mean(per))
    flops = 40320.0 * 512 * 512 * B          # four 3x3 convolutions per output pixel
    achieved = flops / ((ms - ms_mci) * 1e-3) / 1e12
    return {
        "metric": METRIC, "value": B * 512 * 512 / (ms * 1e-3), "unit": "px/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"MCI x2 (256^2 -> 512^2, RGB) + residual CNN refiner (4 conv3x3, 32 ch, BF16 MFMA), "
                               + (f"trained on {args.pairs} method-generated 512^2 RGB pairs x {args.epochs} epochs, "
                                  f"PSNR on {n_eval} held-out 512^2 images" if train else
                                  "initial weights, throughput only (--workload refiner trains and scores it)"),
                   "batch": B},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": achieved / 2500.0, "traffic": None, "kernel": "refiner forward (4 conv layers)"},
        "images_per_s": {"mci": B / (ms_mci * 1e-3), "mci_plus_cnn": B / (ms * 1e-3)},
        "psnr_db": {"mci": p_mci, "mci_plus_cnn": p_ref, "gain": p_ref - p_mci, "images": n_eval,
                    "refined_fraction": frac} if train else None,
        "training": {"pairs": args.pairs, "size": 512, "epochs": args.epochs, "steps": args.epochs * (args.pairs // 16),
                     "seconds": t_train} if train else None,
        "fallback_tau": tau, "train_loss": hist[-1][1] if hist else None, "wall_s": wall,
    }


def main():
    args = parse()
    if args.write_traffic:
        write_traffic(*args.write_traffic)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (every signal and image is independent, "
              "so a batch would shard by contiguous ranges with no collective). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.workload == "batched1d":
        res = bench_batched1d(args, torch)
        if not args.no_2d:
            # the metric's 2-D part: x2 and x4 on 256 images each, same steps and warm-up, each
            # with its own roofline, oracle baseline, errors and PSNR
            sub = copy.copy(args)
            sub.batch = 0
            sub.cpu_sample = 0
            for s in (2, 4):
                log(f"2-D x{s} workload")
                r2 = bench_sisr(sub, torch, s)
                _extrapolate_cpu(r2)
                for key in ("metric", "n_gpus", "steps", "warmup", "higher_is_better", "scaling", "vs_baseline",
                            "data"):
                    r2.pop(key, None)
                res[f"sisr{s}"] = r2
        if not args.no_uneven:
            # not part of the metric: the uneven batch, measured in the same run; a failure
            # here is recorded in the line instead of losing the line
            sub = copy.copy(args)
            sub.batch = 0
            sub.cpu_sample = 0
            log("uneven-batch workload")
            try:
                ru = bench_uneven(sub, torch)
                _extrapolate_cpu(ru)
                for key in ("metric", "n_gpus", "steps", "warmup", "higher_is_better", "scaling", "vs_baseline",
                            "data", "classes"):
                    ru.pop(key, None)   # the per-class table stays in the standalone run's line
                res["uneven"] = ru
            except Exception as e:  # noqa: BLE001
                res["uneven"] = {"error": f"{type(e).__name__}: {e}"}
        if not args.no_refiner:
            # not part of the metric: the refiner's forward throughput at batch 64 (MCI x2 + CNN on
            # 512^2 RGB images); training and PSNR are --workload refiner's
            sub = copy.copy(args)
            sub.batch = 0
            log("refiner forward (throughput only)")
            try:
                rr = bench_refiner(sub, torch, train=False)
                for key in ("metric", "n_gpus", "steps", "warmup", "higher_is_better", "scaling", "vs_baseline",
                            "data", "psnr_db", "training", "fallback_tau", "train_loss"):
                    rr.pop(key, None)
                res["refiner_forward"] = rr
            except Exception as e:  # noqa: BLE001
                res["refiner_forward"] = {"error": f"{type(e).__name__}: {e}"}
    elif args.workload == "refiner":
        res = bench_refiner(args, torch)
    elif args.workload == "uneven":
        res = bench_uneven(args, torch)
    elif args.workload == "offgrid":
        res = bench_offgrid(args, torch)
    elif args.workload == "errsel":
        res = bench_errsel(args, torch)
    elif args.workload == "sisr3":
        # the setting of the paper's super-resolution experiments: x3 with {x, Dx, D2x} per axis
        res = bench_sisr(args, torch, 3, M=3, HR=384)
    else:
        res = bench_sisr(args, torch, 2 if args.workload == "sisr2" else 4)
    _extrapolate_cpu(res)
    print(json.dumps(res), flush=True)


def _extrapolate_cpu(res):
    cpu = res.get("cpu_baseline")
    if cpu and cpu.get("unit") == res.get("unit") and cpu.get("value"):
        # the oracle's time for one whole step of the workload, extrapolated from its sample
        cpu["full_step_s_extrapolated"] = res["value"] * res["ms_per_step"] * 1e-3 / cpu["value"]


if __name__ == "__main__":
    main()
