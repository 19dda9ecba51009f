"""Training and evaluation of the learned denoiser on pairs the compositor
itself generates: a few-frame accumulation (n = 1, 2, 4, 8) as input and a
many-frame accumulation as target, all produced by dfb_composite_frame with
DFB_ACCUMULATE and read through dfb_denoiser_frame_input.  Every step of the
network (forward, backward, Adam) runs in the HIP library; this module only
orchestrates: it picks crops, calls the C ABI and keeps score.

    python -m paper_2305_07083_amd.denoise_train [--scenes S] [--steps N] [--json out.json]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

if __package__ in (None, ""):  # run as a script: make the package importable
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import paper_2305_07083_amd as dfb  # noqa: E402

N_INPUTS = (1, 2, 4, 8)
SIGMA = 0.2


def _torch():
    import torch
    return torch


def _scene(args):
    import workloads
    seed, az, el, size = args
    return workloads.c5(seed=seed, width=size, height=size, azimuth=az, elevation=el)


def make_scenes(seeds, size=2048, rng_seed=1000, processes=8, test_view=False):
    """Scene s: c5 geometry with a random view (azimuth U[0,360), elevation
    U[10,60] from PCG64(rng_seed) in seed order); the test view is 30/25."""
    rng = np.random.Generator(np.random.PCG64(rng_seed))
    jobs = []
    for s in seeds:
        az, el = float(rng.uniform(0, 360)), float(rng.uniform(10, 60))
        jobs.append((s, 30.0, 25.0, size) if test_view else (s, az, el, size))
    if processes > 1 and len(jobs) > 1:
        # fresh interpreters (spawn): the caller may already hold a GPU context
        import multiprocessing
        from concurrent.futures import ProcessPoolExecutor
        ctx = multiprocessing.get_context("spawn")
        with ProcessPoolExecutor(min(processes, len(jobs)), mp_context=ctx) as ex:
            return list(ex.map(_scene, jobs))
    return [_scene(j) for j in jobs]


class Accumulation:
    """A compositor accumulating noisy frames of one scene on the device."""

    def __init__(self, frame, sigma, seed, stream=0):
        import workloads
        self.f = frame
        self.noise = workloads.DeviceNoise(frame, sigma, seed)
        cfg = dfb.make_config(frame.width, frame.height, 64, work=32, waves=4)
        self.c = dfb.Compositor(cfg, stream)
        self.n = 0

    def add(self, frames=1):
        for _ in range(frames):
            x = self.noise.next()
            self.c.set_fragments(x, x.shape[0], self.f.layers, self.f.expected)
            self.c.composite(accumulate=True)
            self.n += 1

    def network_input(self):
        torch = _torch()
        t = torch.empty((self.f.height, self.f.width, 6), dtype=torch.float32, device="cuda")
        dfb.dfb_denoiser_frame_input(self.c.h, t)
        return t

    def tile_variance(self):
        return self.c.read(dfb.DFB_BUF_TILE_VARIANCE)

    def close(self):
        self.c.close()


def build_pairs(scenes, n_target=256, seed=1):
    """For each scene: network inputs after 1, 2, 4, 8 frames and the RGB of
    the n_target-frame mean as target; also the largest tile variance seen at
    each n (the fallback threshold is derived from it)."""
    torch = _torch()
    pairs, vmax = [], {n: 0.0 for n in N_INPUTS}
    for i, f in enumerate(scenes):
        acc = Accumulation(f, SIGMA, seed * 7919 + i)
        ins = {}
        while acc.n < n_target:
            acc.add()
            if acc.n in N_INPUTS:
                ins[acc.n] = acc.network_input()
                if acc.n >= 2:
                    vmax[acc.n] = max(vmax[acc.n], float(np.max(acc.tile_variance())))
        target = acc.network_input()[..., :3].contiguous()
        acc.close()
        pairs.append((ins, target))
        torch.cuda.synchronize()
    return pairs, vmax


def train(net, pairs, steps, batch=8, crop=128, lr=1e-3, seed=0, log=None):
    """Adam on random crops (scene, n, position uniform; n in 1, 2, 4, 8);
    learning rate cosine-decayed from lr to lr/20."""
    torch = _torch()
    rng = np.random.Generator(np.random.PCG64(seed))
    H, W = pairs[0][1].shape[:2]
    xin = torch.empty((batch, crop, crop, 6), dtype=torch.float32, device="cuda")
    tgt = torch.empty((batch, crop, crop, 3), dtype=torch.float32, device="cuda")
    losses = []
    t0 = time.perf_counter()
    for step in range(steps):
        for b in range(batch):
            s = int(rng.integers(len(pairs)))
            n = N_INPUTS[int(rng.integers(len(N_INPUTS)))]
            y = int(rng.integers(0, (H - crop) // 4 + 1)) * 4
            x = int(rng.integers(0, (W - crop) // 4 + 1)) * 4
            xin[b].copy_(pairs[s][0][n][y:y + crop, x:x + crop])
            tgt[b].copy_(pairs[s][1][y:y + crop, x:x + crop])
        cur = lr * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * step / max(1, steps))))
        want = (step % 50 == 0) or step == steps - 1
        loss = dfb.dfb_denoiser_train_step(net, xin, tgt, batch, crop, crop, cur, True, want_loss=want)
        if want:
            losses.append((step, loss))
            if log:
                log("step %d loss %.6f lr %.2e %.1f s" % (step, loss, cur, time.perf_counter() - t0))
    torch.cuda.synchronize()
    return losses, time.perf_counter() - t0


def psnr(img, ref):
    """10 log10(1 / MSE) over pixels and RGB, linear, unclamped, peak 1."""
    d = np.asarray(img, np.float64)[..., :3] - np.asarray(ref, np.float64)[..., :3]
    return 10.0 * math.log10(1.0 / float(np.mean(d * d)))


def gpu_reference(frame):
    """The noise-free composite (the limit of the accumulation) from the GPU
    compositor, tile-major [T, P, 4]."""
    torch = _torch()
    cfg = dfb.make_config(frame.width, frame.height, 64, work=32, waves=4, flags=dfb.DFB_KEEP_FINISHED)
    with dfb.Compositor(cfg, 0) as c:
        c.set_fragments(torch.from_numpy(frame.frag).cuda(), frame.frag.shape[0], frame.layers, frame.expected)
        c.composite()
        return c.read(dfb.DFB_BUF_FINISHED_F32)


def evaluate(net, frame, vmax, ref, n_plain=64, seed=12345, tau_factor=2.0):
    """Plain-accumulation PSNR at n = 1..n_plain (powers of two) and denoised
    PSNR at n = 1, 2, 4, 8 against ``ref`` (noise-free composite, [T, P, 4]);
    frames-to-PSNR = smallest n with denoised PSNR >= plain PSNR at n_plain;
    device times of n frames + denoise vs n_plain plain frames."""
    torch = _torch()
    res = {"plain": {}, "denoised": {}, "fallback_tiles": {}, "tau": {}}
    acc = Accumulation(frame, SIGMA, seed)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for n in range(1, n_plain + 1):
        acc.add()
        if n & (n - 1) == 0:
            res["plain"][n] = psnr(acc.c.read(dfb.DFB_BUF_ACCUM_F32), ref)
        if n in N_INPUTS:
            tau = tau_factor * vmax[n] if n >= 2 else float("inf")
            dfb.dfb_denoise(acc.c.h, net, tau)
            den = acc.c.read(dfb.DFB_BUF_DENOISED_F32)
            res["denoised"][n] = psnr(den, ref)
            res["tau"][n] = tau
            res["fallback_tiles"][n] = int(np.sum(acc.tile_variance() > tau)) if n >= 2 else 0
    acc.close()
    target = res["plain"][n_plain]
    res["frames_to_psnr"] = next((n for n in N_INPUTS if res["denoised"][n] >= target), None)
    # timing (device): n_plain accumulating frames vs n frames + denoise
    acc = Accumulation(frame, SIGMA, seed + 1)
    acc.add(2)
    torch.cuda.synchronize()
    ev0.record()
    acc.add(n_plain)
    ev1.record()
    torch.cuda.synchronize()
    res["ms_plain"] = ev0.elapsed_time(ev1)
    res["ms_denoised"] = {}
    for n in N_INPUTS:
        acc.c.reset()
        torch.cuda.synchronize()
        ev0.record()
        acc.add(n)
        dfb.dfb_denoise(acc.c.h, net, float("inf"))
        ev1.record()
        torch.cuda.synchronize()
        res["ms_denoised"][n] = ev0.elapsed_time(ev1)
    # the same without the per-frame noise draw of this harness: four noisy
    # frames drawn up front and rotated, so only the compositor (and the
    # denoiser) run in the timed region
    frames = [acc.noise.next().clone() for _ in range(4)]

    def composite_only(n):
        for i in range(n):
            x = frames[i % 4]
            acc.c.set_fragments(x, x.shape[0], acc.f.layers, acc.f.expected)
            acc.c.composite(accumulate=True)

    acc.c.reset()
    composite_only(2)
    torch.cuda.synchronize()
    ev0.record()
    composite_only(n_plain)
    ev1.record()
    torch.cuda.synchronize()
    res["ms_plain_compositor_only"] = ev0.elapsed_time(ev1)
    res["ms_denoised_compositor_only"] = {}
    for n in N_INPUTS:
        acc.c.reset()
        torch.cuda.synchronize()
        ev0.record()
        composite_only(n)
        dfb.dfb_denoise(acc.c.h, net, float("inf"))
        ev1.record()
        torch.cuda.synchronize()
        res["ms_denoised_compositor_only"][n] = ev0.elapsed_time(ev1)
    del frames
    # denoise alone
    ev0.record()
    for _ in range(5):
        dfb.dfb_denoise(acc.c.h, net, float("inf"))
    ev1.record()
    torch.cuda.synchronize()
    res["ms_denoise_only"] = ev0.elapsed_time(ev1) / 5
    acc.close()
    return res


def run(scenes=16, steps=1500, batch=8, crop=128, size=2048, log=print):
    # scenes first: the worker processes start before this process touches the GPU
    t0 = time.perf_counter()
    train_frames = make_scenes(range(1, scenes + 1), size=size)
    test_frame = make_scenes([0], size=size, test_view=True)[0]
    log("scenes generated in %.1f s" % (time.perf_counter() - t0))
    torch = _torch()
    dfb.load()
    t1 = time.perf_counter()
    pairs, vmax = build_pairs(train_frames)
    log("pairs built in %.1f s; max tile variance %s" % (time.perf_counter() - t1, vmax))
    net = dfb.Denoiser(max(batch * crop * crop, size * size), seed=0)
    try:
        losses, t_train = train(net.net, pairs, steps, batch, crop, log=log)
        del pairs
        torch.cuda.empty_cache()
        ref = gpu_reference(test_frame)
        res = evaluate(net.net, test_frame, vmax, ref)
        res.update({"train_seconds": t_train, "steps": steps, "batch": batch, "crop": crop,
                    "scenes": scenes, "loss_curve": losses, "vmax": vmax})
        return res, net, test_frame
    except BaseException:
        net.close()
        raise


def time_kernels(size=2048, passes=5, steps=10, batch=8, crop=128, log=print):
    """Device time of the network alone, randomly initialised: forward passes
    on a random 1 x size x size x 6 input, then training steps on random
    batch x crop x crop crops (3 untimed warm-up calls each)."""
    torch = _torch()
    dfb.load()
    res = {}
    with dfb.Denoiser(max(size * size, batch * crop * crop), seed=0) as net:
        x = torch.rand((1, size, size, 6), device="cuda")
        out = torch.empty((1, size, size, 3), device="cuda")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(3):
            dfb.dfb_denoiser_forward(net.net, x, out, 1, size, size)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(passes):
            dfb.dfb_denoiser_forward(net.net, x, out, 1, size, size)
        e1.record()
        torch.cuda.synchronize()
        res["ms_forward"] = e0.elapsed_time(e1) / passes
        xin = torch.rand((batch, crop, crop, 6), device="cuda")
        tgt = torch.rand((batch, crop, crop, 3), device="cuda")
        for _ in range(3):
            dfb.dfb_denoiser_train_step(net.net, xin, tgt, batch, crop, crop, 1e-3, True, want_loss=False)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            dfb.dfb_denoiser_train_step(net.net, xin, tgt, batch, crop, crop, 1e-3, True, want_loss=False)
        e1.record()
        torch.cuda.synchronize()
        res["ms_train_step"] = e0.elapsed_time(e1) / steps
    log("forward %dx%d: %.3f ms; train step %dx%dx%d: %.3f ms" % (size, size, res["ms_forward"], batch, crop, crop,
                                                                 res["ms_train_step"]))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--scenes", type=int, default=16)
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--crop", type=int, default=128)
    ap.add_argument("--json", default=None)
    ap.add_argument("--time-only", action="store_true",
                    help="only time the network's kernels (random weights, random inputs)")
    a = ap.parse_args()
    if a.time_only:
        time_kernels(log=lambda m: print(m, flush=True))
        return
    res, net, _ = run(a.scenes, a.steps, a.batch, a.crop, log=lambda m: print(m, flush=True))
    net.close()
    txt = json.dumps(res, default=float)
    print(txt, flush=True)
    if a.json:
        with open(a.json, "w") as fh:
            fh.write(txt)


if __name__ == "__main__":
    main()
