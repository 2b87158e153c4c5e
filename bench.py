"""Benchmark of the folded-data radiometer map-making hot path on one MI355X.

One step = the whole path for one folded day of one baseline:
  make_maps (dirty map X and Fisher diagonal Gam for every bin and pixel)
  + reduce_band over the full band (broadband Xbb, Gbb).
Inputs (seeds gamma/tau, CSD C, weights w) are resident in HBM before timing.

Prints ONE JSON line with the metric (map terms/s, t * f * pixel, for X + Gam),
the dirty-map kernel's roofline, per-step latency percentiles and a CPU
baseline (the FP64 oracle timed on a bounded sample of the same workload).
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

import synth  # noqa: E402

PEAK_FP32_VECTOR_TFLOPS = 157.3  # MI355X published fp32 vector peak
X_FLOPS_PER_TERM = 10            # complex rotation 6 + Re(y z) accumulation 4
CPU_BASELINE_TARGET_S = 15.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_inputs(sg, torch, wl, dev):
    tg, fgd = wl.tgrid, wl.fgrid
    gamma, tau = sg.build_geometry(synth.baseline_sites(wl.baseline), wl.nside,
                                   sg.TGrid(tg.nt, tg.t0, tg.stride, tg.dur), device=dev)
    f = fgd.freqs()
    C = synth.noise_csd(wl.noise_seed, tg.nt, f, dtype=np.complex128)
    if wl.src_pix:
        src = list(wl.src_pix)
        if wl.nside != 32:
            c32, _ = sg.healpix_centres(32, device=dev)
            cN, _ = sg.healpix_centres(wl.nside, device=dev)
            src = [int(torch.argmax(cN @ c32[p])) for p in src]
        for p, A in zip(src, wl.src_amp):
            synth.add_point_source(C, f, A, gamma[:, p].double().cpu().numpy(), tau[:, p].cpu().numpy())
    w = synth.weights(f, synth.segment_scale(tg.nt, wl.nonstationary_seed)).astype(np.float32)
    Cd = torch.from_numpy(C.astype(np.complex64)).to(dev)
    wd = torch.from_numpy(w).to(dev)
    Hd = torch.from_numpy(synth.spectrum_H(f).astype(np.float32)).to(dev)
    torch.cuda.synchronize()
    return dict(C=Cd, w=wd, H=Hd, gamma=gamma, tau=tau,
                C_host=C.astype(np.complex64).astype(np.complex128), w_host=w.astype(np.float64))


def cpu_baseline(inp, wl, target_s=CPU_BASELINE_TARGET_S):
    """Time the FP64 oracle on a bounded, deterministic sample of the workload."""
    import oracle

    oracle.build()
    tg, fgd = wl.tgrid, wl.fgrid
    npix = 12 * wl.nside ** 2
    gh = inp["gamma"].cpu().numpy()
    th = inp["tau"].cpu().numpy()
    threads = oracle.default_threads()
    rng = np.random.default_rng(77)
    # calibrate on a small sample, then size the timed sample for ~target_s
    n0 = 2000
    cols = rng.integers(0, fgd.nf, n0)
    pix = rng.integers(0, npix, n0)
    t0 = time.perf_counter()
    oracle.maps_at(inp["C_host"], inp["w_host"], fgd.f0, fgd.df, fgd.k0, gh, th, cols, pix, nthreads=threads)
    dt0 = time.perf_counter() - t0
    n = int(max(n0, min(4e7, n0 * target_s / max(dt0, 1e-3))))
    cols = rng.integers(0, fgd.nf, n)
    pix = rng.integers(0, npix, n)
    t0 = time.perf_counter()
    oracle.maps_at(inp["C_host"], inp["w_host"], fgd.f0, fgd.df, fgd.k0, gh, th, cols, pix, nthreads=threads)
    dt = time.perf_counter() - t0
    terms = n * tg.nt
    return {"value": terms / dt, "unit": "terms/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} random (bin, pixel) outputs x all {tg.nt} segments (X and Gam), "
                      f"{dt:.1f} s wall on {threads} threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=2, help="2: full band nside 32; 3: full band nside 64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the path shards by "
              f"pixel or frequency with no collective; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1803_08285_amd as sg

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    wl = synth.workload(args.workload)
    tg, fgd = wl.tgrid, wl.fgrid
    npix = 12 * wl.nside ** 2
    log(f"workload {wl.name}: nt={tg.nt} nf={fgd.nf} npix={npix}")
    inp = make_inputs(sg, torch, wl, dev)
    X = torch.empty((fgd.nf, npix), dtype=torch.float32, device=dev)
    G = torch.empty_like(X)
    Xbb = torch.empty(npix, dtype=torch.float32, device=dev)
    Gbb = torch.empty_like(Xbb)
    ws = sg.make_workspace(tg.nt, fgd.nf, npix, True, device=dev)
    fg = sg.FGrid(fgd.f0, fgd.df)

    def step(evs=None):
        if evs:
            evs[0].record()
        sg.make_maps(inp["C"], inp["w"], fg, fgd.k0, inp["gamma"], inp["tau"], want_gamma=False, out=(X, None))
        if evs:
            evs[1].record()
        sg.make_maps(inp["C"], inp["w"], fg, fgd.k0, inp["gamma"], inp["tau"], want_x=False, out=(None, G),
                     workspace=ws)
        if evs:
            evs[2].record()
        sg.reduce_band(X, G, inp["H"], 0, fgd.nf, out=(Xbb, Gbb))
        if evs:
            evs[3].record()

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {wall:.3f} s")
    t_x = np.array([e[0].elapsed_time(e[1]) for e in evs])
    t_g = np.array([e[1].elapsed_time(e[2]) for e in evs])
    t_b = np.array([e[2].elapsed_time(e[3]) for e in evs])
    t_step = np.array([e[0].elapsed_time(e[3]) for e in evs])
    ms_per_step = wall * 1e3 / args.steps
    terms = tg.nt * fgd.nf * npix
    x_tflops = X_FLOPS_PER_TERM * terms / (t_x.mean() * 1e-3) / 1e12

    if args.copy_calib_mib:
        nbytes = args.copy_calib_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {nbytes} bytes read, {nbytes} bytes written")
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on the host cores")
        cpu = cpu_baseline(inp, wl)

    out = {
        "metric": "map terms/s (t*f*pix) for X+Gamma",
        "value": terms / (ms_per_step * 1e-3),
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded noise model + injected point sources)",
        "config": {"workload": wl.name, "baseline": wl.baseline, "nt": tg.nt, "nf": fgd.nf, "nside": wl.nside,
                   "npix": npix, "f0_hz": fgd.f0, "df_hz": fgd.df, "terms_per_step": terms,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "kernel": "dirty_map_kernel<float, pair>",
                     "achieved": x_tflops, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": x_tflops / PEAK_FP32_VECTOR_TFLOPS, "traffic": None,
                     "flops_per_term": X_FLOPS_PER_TERM, "launch_ms": float(t_x.mean())},
        "phases_ms": {"dirty_map": float(t_x.mean()), "beam": float(t_g.mean()), "band": float(t_b.mean())},
        "latency_ms": {"p50": float(np.percentile(t_step, 50)), "p99": float(np.percentile(t_step, 99))},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
