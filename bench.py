"""Throughput of the per-tile sort-last compositing path on one MI355X.

One step = one frame of the 2048x2048, 64x64-tile, 4x4x4-brick (64 ranks)
fragment set through the whole path in one persistent launch: per-pixel
depth sort, front-to-back over with the background, Welford accumulation,
per-tile variance and RGBA8 tonemapping.  Inputs are resident in HBM before
the timed region; four copies rotate so the 555 MB working set cannot stay in
the 256 MB last-level cache.  Prints one JSON line.

The line also carries the learned part of the metric ("denoise"): frames to
reach the 64-frame plain PSNR with the denoiser, trained on the GPU by the
library's own kernels on compositor-generated pairs.

  python bench.py [--steps K] [--warmup W] [--workload c2|c3|c3f16|c1] [--no-cpu] [--no-denoise]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "composited fragments/s + HBM GB/s % peak; frames-to-PSNR denoised vs plain"
HBM_PEAK_GBPS = 8000.0


def log(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def median_mad(xs):
    """Median and median absolute deviation (unscaled), the statistics the
    paper reports its timings with."""
    import numpy as np
    a = np.asarray(xs, dtype=np.float64)
    med = float(np.median(a))
    return med, float(np.median(np.abs(a - med)))


def cpu_model():
    """The host CPU's model name as lscpu reports it (else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c3f16", "c4"])
    ap.add_argument("--copies", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--plain", action="store_true", help="composite only (no accumulation)")
    ap.add_argument("--no-denoise", action="store_true",
                    help="skip training / evaluating the denoiser (frames-to-PSNR part of the metric)")
    ap.add_argument("--denoise-scenes", type=int, default=16)
    ap.add_argument("--denoise-steps", type=int, default=1000)
    ap.add_argument("--no-ops", action="store_true",
                    help="skip the list / average tile-operation legs")
    ap.add_argument("--no-other", action="store_true",
                    help="skip the 4096x1024 (fp32, fp16) and 8192x8192 sort-path legs")
    ap.add_argument("--event-frames", type=int, default=30,
                    help="frames of the separate timing pass with HIP events around every frame kernel")
    ap.add_argument("--time-every", type=int, default=5,
                    help="HIP events around the frame kernel of every n-th timed headline frame "
                         "(each timed frame carries two event records, ~3.5 us each)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the run, copy 1 GiB device to device (the reference kernel for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


KERNEL_SOURCES = ["dfb_kernels.hip", "dfb_internal.h", "sortnet.h"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2305_07083_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_counter_profile(path):
    """The ``key: value`` lines of a committed rocprofv3 counter summary
    (comment lines skipped), or None if the file is missing or its counters
    were taken on another kernel source than the current one."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    return kv if kv.get("kernel_source_hash") == kernel_source_hash() else None


def counter_bytes(kv, prefix):
    """HBM bytes per launch: scaled FETCH_SIZE + WRITE_SIZE (KiB per dispatch)."""
    if kv is None or prefix + "fetch_kib_per_dispatch" not in kv:
        return None
    fetch = float(kv[prefix + "fetch_kib_per_dispatch"]) * float(kv["fetch_scale"])
    write = float(kv[prefix + "write_kib_per_dispatch"]) * float(kv["write_scale"])
    return (fetch + write) * 1024.0


def measured_traffic(workload, accumulate):
    """HBM bytes per frame-kernel launch from the committed rocprofv3 counter
    summary of this workload, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "frame_kernel_%s_%s_counters.txt"
                        % (workload, "acc" if accumulate else "plain"))
    return counter_bytes(read_counter_profile(path), "")


def measured_leg_traffic(profile, leg):
    """HBM bytes per launch of one leg's kernel (``leg``_fetch / _write keys)
    from a committed counter summary (current kernel source only)."""
    return counter_bytes(read_counter_profile(os.path.join(ROOT, "profiles", profile)), leg + "_")


def measured_op_traffic(op):
    """The tile-op legs (list, average, and the per-pixel sort of the same
    brick frame)."""
    return measured_leg_traffic("frame_kernel_tile_ops_2048_counters.txt", op)


BF16_PEAK_TFLOPS = 2500.0


def denoiser_flops_per_pixel():
    """Multiply-adds x 2 of one forward pass per full-resolution pixel."""
    import paper_2305_07083_amd as dfb
    f = sum(2 * 9 * ci * co / 4 ** lvl for _, ci, co, lvl in dfb.UNET_CONV3)
    return f + 2 * 32 * 3


UP_LAYERS = ("up2", "up1")         # read their input through the 2x up-sampling
POOL_LAYERS = ("enc1b", "enc2b")   # also write the 2x2-pooled map


def denoiser_roofline_us(width, height):
    """Lower bound of one dfb_denoise call: per conv layer max(flops / BF16
    peak, algorithmic bytes / HBM peak), plus the HBM time of the glue
    (frame -> input, bf16 packing, 1x1 output conv, fallback selection +
    RGBA8).  Algorithmic bytes of a layer: its input map read once (bf16,
    the 6 input channels stored as 8), its output (and pooled) map written
    once."""
    import paper_2305_07083_amd as dfb
    P0 = width * height
    t = 0.0
    flops = 0.0
    nbytes = 0.0
    for name, ci, co, lvl in dfb.UNET_CONV3:
        px = P0 / 4 ** lvl
        ci_store = 8 if ci == 6 else ci
        rb = (px / 4 if name in UP_LAYERS else px) * ci_store * 2
        wb = px * co * 2 + (px / 4 * co * 2 if name in POOL_LAYERS else 0)
        fl = 2.0 * 9 * ci * co * px
        t += max(fl / (BF16_PEAK_TFLOPS * 1e12), (rb + wb) / (HBM_PEAK_GBPS * 1e9))
        flops += fl
        nbytes += rb + wb
    glue = P0 * ((16 + 24) + (24 + 16) + (64 + 24 + 12) + (16 + 12 + 16 + 4))
    t += glue / (HBM_PEAK_GBPS * 1e9)
    return t * 1e6, flops, nbytes + glue


def denoise_leg(scenes, steps):
    """Frames-to-PSNR of the learned denoiser vs plain accumulation on the
    2048x2048 smooth-field brick scene (sigma 0.2): train on compositor pairs
    from ``scenes`` other views, evaluate on the 30/25 view.  PSNR reference:
    the noise-free composite from the GPU compositor (the limit of the
    accumulation; the tests pin it to the FP64 oracle)."""
    from paper_2305_07083_amd import denoise_train as dt
    res, net, test = dt.run(scenes=scenes, steps=steps, log=lambda m: print(m, file=sys.stderr, flush=True))
    net.close()
    flops = denoiser_flops_per_pixel() * test.width * test.height
    tflops = flops / (res["ms_denoise_only"] * 1e-3) / 1e12
    roof_us, _, roof_bytes = denoiser_roofline_us(test.width, test.height)
    return {
        "workload": "2048x2048 frame, 4x4x4 bricks, spatially correlated alpha/colour (16 px), colour noise "
                    "sigma 0.2; 3-level U-Net, 32 base channels, BF16 MFMA, FP32 accumulate",
        "plain_psnr_db": {int(k): v for k, v in res["plain"].items()},
        "denoised_psnr_db": {int(k): v for k, v in res["denoised"].items()},
        "frames_to_psnr": res["frames_to_psnr"],
        "target": "denoised PSNR >= plain PSNR after 64 frames",
        "ms_64_plain_frames": res["ms_plain"],
        "ms_n_frames_plus_denoise": {int(k): v for k, v in res["ms_denoised"].items()},
        "timing_note": "ms_64_plain_frames and ms_n_frames_plus_denoise include this harness's device "
                       "noise draw per frame; the *_compositor_only figures rotate 4 frames drawn up front",
        "ms_64_plain_frames_compositor_only": res["ms_plain_compositor_only"],
        "ms_n_frames_plus_denoise_compositor_only": {int(k): v for k, v in
                                                     res["ms_denoised_compositor_only"].items()},
        "ms_denoise_forward": res["ms_denoise_only"],
        "denoise_roofline": {"bound": "per layer: mfma (bf16) or hbm, whichever is slower",
                             "roofline_ms": roof_us * 1e-3, "achieved_ms": res["ms_denoise_only"],
                             "frac": roof_us * 1e-3 / res["ms_denoise_only"],
                             "flops_per_launch": flops, "algorithmic_bytes_per_launch": roof_bytes,
                             "mfma_tflops": tflops, "mfma_frac": tflops / BF16_PEAK_TFLOPS},
        "fallback_tiles": {int(k): v for k, v in res["fallback_tiles"].items()},
        "train": {"scenes": scenes, "steps": steps, "batch": res["batch"], "crop": res["crop"],
                  "seconds": res["train_seconds"], "final_loss": res["loss_curve"][-1][1]},
    }


class DeviceFrame:
    """The 8192x8192 heavy-tailed frame: layer list on the host, fragment
    values drawn on the device (57.6 GB fp32 does not fit host memory)."""

    def __init__(self):
        import workloads
        self.width = self.height = 8192
        self.tile_w = self.tile_h = 128
        self.layers, K = workloads.zipf_layout(8192, 8192, 128, 512, 1.2, 512, seed=0)
        self.expected = K.astype("int32")
        self.frag = None

    @property
    def n_tiles(self):
        return 64 * 64

    @property
    def P(self):
        return 128 * 128

    @property
    def n_fragments(self):
        return len(self.layers) * self.P


def make_frame(name):
    import numpy as np
    import workloads
    if name == "c4":
        return DeviceFrame(), ("8192x8192 frame, 128x128 tiles, 512 ranks, truncated Zipf(1.2) layers per tile "
                               "(1..512), fp32, work unit and waves autotuned")
    if name == "c1":
        f = workloads.c1()
        desc = "256x256 frame, 64x64 tiles, 4 ranks on every tile, fp32"
    elif name == "c2":
        f = workloads.c2()
        desc = "2048x2048 frame, 64x64 tiles, 4x4x4 bricks (64 ranks), fp32"
    else:
        f = workloads.c3()
        desc = "4096x1024 frame, 64x64 tiles, 8x8x4 bricks (256 ranks), fp32"
        if name == "c3f16":
            f = f.as_dtype(np.float16)
            desc = desc.replace("fp32", "fp16")
    return f, desc


def time_frames(dfb, torch, f, op, copies, steps, warmup):
    """Plain frames (composite + RGBA8) of ``f`` with tile operation ``op``,
    autotuned; returns (kernel ms from the HIP events around the frame kernel, wall ms per frame,
    launch info)."""
    cfg = dfb.make_config(f.width, f.height, f.tile_w, f.tile_h, work=0, waves=0, op=op)
    n_blocks = copies[0].shape[0]
    with dfb.Compositor(cfg, torch.cuda.current_stream().cuda_stream) as c:
        c.set_fragments(copies[0], n_blocks, f.layers, f.expected)
        c.composite()
        for i in range(warmup):
            c.set_fragments(copies[i % len(copies)], n_blocks, f.layers, f.expected)
            c.composite()
        torch.cuda.synchronize()
        dfb.dfb_set_timing(c.h, True)
        t0 = time.perf_counter()
        for i in range(steps):
            c.set_fragments(copies[i % len(copies)], n_blocks, f.layers, f.expected)
            c.composite()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps * 1e3
        return dfb.dfb_kernel_ms(c.h), wall, c.info()


def tile_ops_leg(dfb, torch, steps=30, warmup=5, copies=4):
    """The other tile operations on full-size frames, plain frames with RGBA8
    output: the 2048x2048 brick frame as a generation list (list operation)
    next to the same frame through the per-pixel sort, and redundant renders
    of a 2048x2048 frame (U{1..8} per tile) through the averaging operation.
    Algorithmic bytes per launch: RGBA of every fragment (the list and
    average read no depth; the sort reads RGBA + depth), 4 B per output
    pixel, the layer table."""
    import workloads
    out = {}
    legs = [("list", workloads.bricks_2048_list(), dfb.DFB_OP_LIST, 16,
             "2048x2048, 64x64 tiles, 4x4x4 bricks as a back-to-front generation list, fp32"),
            ("alpha_blend_same_frame", workloads.c2(), dfb.DFB_OP_ALPHA_BLEND, 20,
             "2048x2048, 64x64 tiles, 4x4x4 bricks, per-pixel sort, fp32"),
            ("average", workloads.redundant_2048(), dfb.DFB_OP_AVERAGE, 16,
             "2048x2048, 64x64 tiles, U{1..8} redundant renders per tile, fp32")]
    for name, f, op, frag_bytes, desc in legs:
        bufs = [torch.from_numpy(f.frag).to("cuda:0") for _ in range(copies)]
        torch.cuda.synchronize()
        kms, wall, info = time_frames(dfb, torch, f, op, bufs, steps, warmup)
        del bufs
        torch.cuda.empty_cache()
        px = f.n_tiles * f.P
        alg = f.n_fragments * frag_bytes + px * 4 + f.n_tiles * 4 + len(f.layers) * 8
        gbps = alg / (kms * 1e-3) / 1e9
        out[name] = {"workload": desc, "fragments_per_frame": f.n_fragments, "kernel_ms": kms,
                     "wall_ms_per_frame": wall, "fragments_per_s": f.n_fragments / (kms * 1e-3),
                     "work_tile": [info.work_w, info.work_h], "waves_per_tile": info.waves_per_tile,
                     "roofline": {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                                  "frac": gbps / HBM_PEAK_GBPS,
                                  "traffic": measured_op_traffic(name),
                                  "algorithmic_bytes_per_launch": alg}}
    return out


def other_workloads_leg(dfb, torch, steps=10, warmup=3, with_cpu=True):
    """The sort path on the other frame shapes, accumulating frames (the
    4096x1024 progressive case, fp32 and fp16) and plain frames (the 8192x8192
    heavy-tailed case), autotuned, 2 rotating copies (1 for the device-drawn
    8192x8192 set).  Algorithmic bytes as for the headline."""
    import numpy as np
    import workloads
    out = {}
    dev = torch.device("cuda:0")
    for name, accumulate in (("c3", True), ("c3f16", True), ("c4", False)):
        log("other workloads: " + name)
        f, desc = make_frame(name)
        if name == "c4":
            copies = [workloads.uniform_values_torch(len(f.layers), f.P, seed=0, device=dev)]
            f16 = False
        else:
            copies = [torch.from_numpy(f.frag).to(dev) for _ in range(2)]
            f16 = f.frag.dtype == np.float16
        torch.cuda.synchronize()
        cfg = dfb.make_config(f.width, f.height, f.tile_w, f.tile_h, work=0, waves=0,
                              dtype=dfb.DFB_F16 if f16 else dfb.DFB_F32)
        n_blocks = copies[0].shape[0]
        with dfb.Compositor(cfg, torch.cuda.current_stream().cuda_stream) as c:
            c.set_fragments(copies[0], n_blocks, f.layers, f.expected)
            c.composite()  # autotune
            for i in range(warmup):
                c.set_fragments(copies[i % len(copies)], n_blocks, f.layers, f.expected)
                c.composite(accumulate=accumulate)
            torch.cuda.synchronize()
            dfb.dfb_set_timing(c.h, True)
            for i in range(steps):
                c.set_fragments(copies[i % len(copies)], n_blocks, f.layers, f.expected)
                c.composite(accumulate=accumulate)
            torch.cuda.synchronize()
            times = dfb.dfb_kernel_times(c.h)
            kms = dfb.dfb_kernel_ms(c.h)
            info = c.info()
        cpu = oracle_subset_baseline(f, copies[0], torch) if (name == "c4" and with_cpu) else None
        del copies
        torch.cuda.empty_cache()
        px = f.n_tiles * f.P
        alg = f.n_fragments * (10 if f16 else 20) + px * (4 + (56 if accumulate else 0)) + f.n_tiles * 4 \
            + len(f.layers) * 8
        gbps = alg / (kms * 1e-3) / 1e9
        out[name] = {"workload": desc + (", composite + accumulate + per-tile variance + RGBA8" if accumulate
                                         else ", composite + RGBA8"),
                     "fragments_per_frame": f.n_fragments, "kernel_ms": kms,
                     "kernel_ms_median": median_mad(times)[0], "kernel_ms_mad": median_mad(times)[1],
                     "timed_frames": len(times),
                     "fragments_per_s": f.n_fragments / (kms * 1e-3),
                     "work_tile": [info.work_w, info.work_h], "waves_per_tile": info.waves_per_tile,
                     "roofline": {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                                  "frac": gbps / HBM_PEAK_GBPS,
                                  "traffic": measured_leg_traffic("frame_kernel_other_workloads_counters.txt", name),
                                  "algorithmic_bytes_per_launch": alg}}
        if cpu is not None:
            out[name]["cpu_baseline"] = cpu
    return out


def assign_samples_ms(dfb, n_tiles=4096, extra=16384, reps=20):
    """Host time of one variance-driven assignment of extra renders over
    n_tiles tiles (the library's host routine, seeded variances)."""
    import numpy as np
    v = np.random.default_rng(5).gamma(2.0, 1e-3, n_tiles).astype(np.float32)
    dfb.dfb_assign_samples_host(v, extra)
    t0 = time.perf_counter()
    for _ in range(reps):
        dfb.dfb_assign_samples_host(v, extra)
    return (time.perf_counter() - t0) / reps * 1e3


def cpu_baseline(f, accumulate, runs=3, run_s=3.0):
    """The FP64 oracle as it stands, on whole frames of the same fragment set
    (composite, then accumulate + variance + tonemap when accumulating):
    ``runs`` runs of at least ``run_s`` seconds on all host cores, and
    ``runs`` single-frame runs on one thread.  Median and MAD of the runs."""
    import numpy as np
    import oracle
    threads = len(os.sched_getaffinity(0))
    mu = np.zeros((f.n_tiles, f.P, 4))
    m2 = np.zeros((f.n_tiles, f.P, 3))

    def one_run(n_threads, min_s):
        mu[...] = 0.0
        m2[...] = 0.0
        frames = 0
        t0 = time.perf_counter()
        while True:
            r = oracle.composite(f.frag, f.layers, f.width, f.height, f.tile_w, f.tile_h,
                                 expected=f.expected, threads=n_threads)
            if accumulate:
                oracle.accumulate(mu, m2, r["rgba"], frames + 1)
                oracle.tile_variance(m2, np.arange(f.n_tiles), f.width, f.height, f.tile_w, f.tile_h, frames + 1)
                oracle.tonemap(mu)
            else:
                oracle.tonemap(r["rgba"])
            frames += 1
            dt = time.perf_counter() - t0
            if dt >= min_s:
                return f.n_fragments * frames / dt, frames, dt

    multi = [one_run(threads, run_s) for _ in range(runs)]
    single = [one_run(1, 0.0) for _ in range(runs)]
    med, mad = median_mad([r[0] for r in multi])
    med1, mad1 = median_mad([r[0] for r in single])
    what = "composite+accumulate+variance+tonemap" if accumulate else "composite+tonemap"
    return {"value": med, "unit": "fragments/s", "cores": threads, "kind": "oracle",
            "sample": "%d runs of %s whole frames of the same fragment set (%d fragments each), %s, on %d "
                      "threads; median of the runs"
                      % (runs, "/".join(str(r[1]) for r in multi), f.n_fragments, what, threads),
            "mad": mad, "runs": [r[0] for r in multi],
            "single_thread": {"value": med1, "mad": mad1, "runs": [r[0] for r in single],
                              "sample": "%d runs of 1 whole frame on 1 thread" % runs},
            "cpu_model": cpu_model()}


def oracle_subset_baseline(f, dev_frag, torch, every=50, runs=3):
    """The FP64 oracle on a K-stratified sample of the 8192x8192 frame's
    tiles: the tiles sorted by layer count, every ``every``-th taken, so the
    sample's layer-count mix follows the frame's.  Their blocks are copied
    from the device (the full 57.6 GB set does not fit host memory) and
    composited + tonemapped on all host cores; fragments/s of the sample
    stands for the whole frame (the oracle's cost per fragment depends on K,
    which the sample spans in proportion)."""
    import numpy as np
    import oracle
    threads = len(os.sched_getaffinity(0))
    counts = np.asarray(f.expected)
    order = np.argsort(counts, kind="stable")
    tiles = np.sort(order[every // 2::every]).astype(np.int32)
    sel = np.isin(f.layers["tile_id"], tiles)
    sub = f.layers[sel].copy()
    idx = torch.from_numpy(sub["block"].astype(np.int64)).to(dev_frag.device)
    host = dev_frag.index_select(0, idx).cpu().numpy()
    del idx
    sub["block"] = np.arange(len(sub))
    n_frag = len(sub) * f.P
    rates = []
    for _ in range(runs):
        t0 = time.perf_counter()
        r = oracle.composite(host, sub, f.width, f.height, f.tile_w, f.tile_h, tiles=tiles, threads=threads)
        oracle.tonemap(r["rgba"])
        rates.append(n_frag / (time.perf_counter() - t0))
    med, mad = median_mad(rates)
    return {"value": med, "unit": "fragments/s", "cores": threads, "kind": "oracle", "mad": mad, "runs": rates,
            "sample": "%d of %d tiles (every %dth by layer count: K %d..%d), %d fragments = %.2f%% of the frame's; "
                      "composite + tonemap, median of %d runs; the whole frame at this rate: %.0f s"
                      % (len(tiles), f.n_tiles, every, int(counts[tiles].min()), int(counts[tiles].max()), n_frag,
                         100.0 * n_frag / f.n_fragments, runs, f.n_fragments / med),
            "cpu_model": cpu_model()}


def c1_latency_leg(dfb, torch, frames=30, warmup=10):
    """The 256x256 uniform frame (4 ranks on every tile, 5.2 MB: cache
    resident, so latency rather than a roofline): per-frame kernel time from
    HIP events on every frame, and the end-to-end latency of one
    dfb_set_fragments + dfb_composite_frame + synchronise from the host."""
    import workloads
    f = workloads.c1()
    buf = torch.from_numpy(f.frag).to("cuda:0")
    cfg = dfb.make_config(f.width, f.height, f.tile_w, f.tile_h, work=0, waves=0)
    with dfb.Compositor(cfg, torch.cuda.current_stream().cuda_stream) as c:
        c.set_fragments(buf, f.frag.shape[0], f.layers, f.expected)
        c.composite()
        for _ in range(warmup):
            c.composite()
        torch.cuda.synchronize()
        dfb.dfb_set_timing(c.h, 1)
        for _ in range(frames):
            c.set_fragments(buf, f.frag.shape[0], f.layers, f.expected)
            c.composite()
        k_med, k_mad = median_mad(dfb.dfb_kernel_times(c.h) * 1e3)
        dfb.dfb_set_timing(c.h, 0)
        lat = []
        for _ in range(frames):
            t0 = time.perf_counter()
            c.set_fragments(buf, f.frag.shape[0], f.layers, f.expected)
            c.composite()
            dfb.dfb_synchronize(c.h)
            lat.append((time.perf_counter() - t0) * 1e6)
        info = c.info()
    l_med, l_mad = median_mad(lat)
    return {"workload": "256x256 frame, 64x64 tiles, 4 ranks on every tile, fp32, composite + RGBA8",
            "fragments_per_frame": f.n_fragments, "kernel_us_median": k_med, "kernel_us_mad": k_mad,
            "end_to_end_us_median": l_med, "end_to_end_us_mad": l_mad, "frames": frames,
            "fragments_per_s": f.n_fragments / (k_med * 1e-6),
            "work_tile": [info.work_w, info.work_h], "waves_per_tile": info.waves_per_tile,
            "note": "5.2 MB working set, cache resident: a latency figure, no roofline claim"}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the per-tile exchange between GPUs is not implemented, "
              "so only --gpus 1 runs", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2305_07083_amd as dfb

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dfb.load()
    f, desc = make_frame(args.workload)
    dev = torch.device("cuda:0")
    if args.workload == "c4":
        import workloads
        copies = [workloads.uniform_values_torch(len(f.layers), f.P, seed=0, device=dev)]
        f16 = False
    else:
        copies = [torch.from_numpy(f.frag).to(dev) for _ in range(max(1, args.copies))]
        f16 = f.frag.dtype == np.float16
    torch.cuda.synchronize()
    cfg = dfb.make_config(f.width, f.height, f.tile_w, f.tile_h, work=0, waves=0,
                          dtype=dfb.DFB_F16 if f16 else dfb.DFB_F32, fmt=dfb.DFB_FMT_RGBA8)
    stream = torch.cuda.current_stream().cuda_stream
    accumulate = not args.plain
    n_blocks = copies[0].shape[0]
    with dfb.Compositor(cfg, stream) as c:
        t_in = time.perf_counter()
        c.set_fragments(copies[0], n_blocks, f.layers, f.expected)   # a new layout: host ingest
        ingest_ms = (time.perf_counter() - t_in) * 1e3
        c.composite(accumulate=False)     # first frame of a new layout: autotunes the launch shape
        torch.cuda.synchronize()
        t_in = time.perf_counter()
        c.set_fragments(copies[1 % len(copies)], n_blocks, f.layers, f.expected)  # same layout
        same_layout_ms = (time.perf_counter() - t_in) * 1e3
        # new layouts in steady state: the arrival order alternates between
        # two permutations, so every call is a new layer list (validation,
        # per-tile table, work list, upload), with frames in flight
        alt = [f.layers, f.layers[::-1].copy()]
        new_layout_ms = []
        for i in range(10):
            t_in = time.perf_counter()
            c.set_fragments(copies[i % len(copies)], n_blocks, alt[(i + 1) % 2], f.expected)
            new_layout_ms.append((time.perf_counter() - t_in) * 1e3)
            c.composite(accumulate=False)
        c.set_fragments(copies[0], n_blocks, f.layers, f.expected)
        torch.cuda.synchronize()
        for i in range(args.warmup):
            c.set_fragments(copies[i % len(copies)], n_blocks, f.layers, f.expected)
            c.composite(accumulate=accumulate)
        torch.cuda.synchronize()
        dfb.dfb_set_timing(c.h, max(1, args.time_every))
        t0 = time.perf_counter()
        for i in range(args.steps):
            c.set_fragments(copies[i % len(copies)], n_blocks, f.layers, f.expected)
            c.composite(accumulate=accumulate)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kernel_ms = dfb.dfb_kernel_ms(c.h)
        info = c.info()
        # a separate timing pass: HIP events around every frame kernel
        dfb.dfb_set_timing(c.h, 1)
        for i in range(args.event_frames):
            c.set_fragments(copies[i % len(copies)], n_blocks, f.layers, f.expected)
            c.composite(accumulate=accumulate)
        ev_ms = dfb.dfb_kernel_times(c.h)
        dfb.dfb_set_timing(c.h, 0)
        # the same frames launched as replays of the handle's frame graphs
        # (one per input copy): wall time per frame, then events around every
        # replay (frame kernel + variance combine)
        for i in range(max(len(copies), 3)):
            c.set_fragments(copies[i % len(copies)], n_blocks, f.layers, f.expected)
            c.composite(accumulate=accumulate, replay=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            c.set_fragments(copies[i % len(copies)], n_blocks, f.layers, f.expected)
            c.composite(accumulate=accumulate, replay=True)
        torch.cuda.synchronize()
        graph_wall = time.perf_counter() - t0
        dfb.dfb_set_timing(c.h, 1)
        for i in range(args.event_frames):
            c.set_fragments(copies[i % len(copies)], n_blocks, f.layers, f.expected)
            c.composite(accumulate=accumulate, replay=True)
        graph_ms = dfb.dfb_kernel_times(c.h)
        dfb.dfb_set_timing(c.h, 0)
    frag_bytes = 10 if f16 else 20
    px = f.n_tiles * f.P
    per_px = 4 + (56 if accumulate else 0)       # RGBA8 out (+ mean and M2 read and written)
    alg_bytes = f.n_fragments * frag_bytes + px * per_px + f.n_tiles * 4 + len(f.layers) * 8
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    ms_per_step = wall / args.steps * 1e3
    value = f.n_fragments * args.steps / wall
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "fragments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16" if f16 else "f32",
        "data": "synthetic",
        "config": {"workload": desc + (", composite + accumulate + per-tile variance + RGBA8" if accumulate
                                       else ", composite + RGBA8"),
                   "fragments_per_frame": f.n_fragments, "layers": len(f.layers),
                   "max_layers_per_tile": int(f.expected.max()),
                   "work_tile": [info.work_w, info.work_h], "waves_per_tile": info.waves_per_tile,
                   "grid": info.grid_size},
        "kernel_ms": kernel_ms,
        "kernel_timing": "HIP events around the frame kernel of 1 in every %d of the %d timed frames"
                         % (max(1, args.time_every), args.steps),
        "kernel_timing_every_frame": {
            "frames": int(len(ev_ms)), "median_ms": median_mad(ev_ms)[0], "mad_ms": median_mad(ev_ms)[1],
            "mean_ms": float(np.mean(ev_ms)),
            "achieved_gbps_median": alg_bytes / (median_mad(ev_ms)[0] * 1e-3) / 1e9,
            "how": "a separate pass after the timed one: HIP events around every frame kernel"},
        "graph_replay": {
            "wall_ms_per_frame": graph_wall / args.steps * 1e3,
            "stream_launch_wall_ms_per_frame": wall / args.steps * 1e3,
            "events_median_ms": median_mad(graph_ms)[0], "events_mad_ms": median_mad(graph_ms)[1],
            "how": "DFB_REPLAY: each frame a hipGraphLaunch of the handle's graph (frame kernel + variance "
                   "combine, one graph per input copy); events bracket the whole graph"},
        "host_ms": {"ingest_new_layout": median_mad(new_layout_ms)[0],
                    "ingest_new_layout_how": "median of 10 dfb_set_fragments calls, each a new layer list "
                                             "(alternating arrival orders), a frame composited after each",
                    "ingest_first_layout": ingest_ms, "set_fragments_same_layout": same_layout_ms,
                    "assign_samples_4096_tiles": assign_samples_ms(dfb)},
        "hbm_gbps_algorithmic": achieved,
        "hbm_frac_of_peak": achieved / HBM_PEAK_GBPS,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": measured_traffic(args.workload, accumulate),
                     "algorithmic_bytes_per_launch": alg_bytes},
    }
    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    log("headline done: %.4f ms per frame, kernel %.4f ms" % (ms_per_step, kernel_ms))
    if not args.no_cpu and args.workload != "c4":
        out["cpu_baseline"] = cpu_baseline(f, accumulate)
        log("cpu baseline done")
    if args.workload == "c2":
        out["c1_latency"] = c1_latency_leg(dfb, torch)
        log("c1 latency done")
    if not args.no_ops and args.workload == "c2":
        out["tile_ops"] = tile_ops_leg(dfb, torch)
        log("tile ops done")
    if not args.no_other and args.workload == "c2":
        del copies
        torch.cuda.empty_cache()
        out["other_workloads"] = other_workloads_leg(dfb, torch, with_cpu=not args.no_cpu)
        log("other workloads done")
    if not args.no_denoise and args.workload == "c2":
        out["denoise"] = denoise_leg(args.denoise_scenes, args.denoise_steps)
        log("denoise done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
