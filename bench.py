"""Benchmark of the folded-data radiometer map-making hot path on one MI355X.

One step = the whole path for one folded day of one baseline: the dirty map X
and the Fisher diagonal Gam for every bin and pixel, and their broadband sums
Xbb, Gbb over the full band (make_maps_band: the band sums are taken inside the
map kernels).
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
PEAK_F16_MFMA_TFLOPS = 2500.0    # MI355X published dense fp16/bf16 matrix peak
X_FLOPS_PER_TERM = 10            # algorithmic: rotation 6 + Re(y z) accumulation 4 (vector form);
                                 # the matrix form's 5-term contraction is also 10 flops per term
# Matrix form as issued: float16 products per term per component x 2 flops x 2
# components / 2 pixels per antipodal pair = 2 x products, by the form the call
# took (four terms: 8 products; five with m = 2 unsplit: 9; split: 11).
ISSUED_FLOPS_PER_TERM = {"mfma4": 16, "mfma5": 18, "mfma5_split": 22}

CPU_BASELINE_TARGET_S = 24.0
# The arithmetic the path computes in: the dirty map as float16 hi + lo products
# on the matrix cores with float64 phase reduction, the beam as bfloat16 hi + lo
# products, both accumulated in float32.
DTYPE_LABEL = "split-f16 (X) / split-bf16 (Gamma) MFMA, f32 accumulate, f64 phase"
# Sources of the matrix-core dirty-map kernel: a recorded HBM traffic figure is
# reported only while these are unchanged since the counters were taken.
X_KERNEL_SOURCES = ("paper_1803_08285_amd/csrc/dirty_map_mfma.hip", "paper_1803_08285_amd/csrc/sgwb_internal.h")


def sources_sha256(paths):
    import hashlib

    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def recorded_traffic(workload: str):
    """HBM bytes per launch of the dirty-map kernel from the committed counter
    summary (FETCH_SIZE x2 + WRITE_SIZE x1, calibrated on a plain copy), or None
    if there is none for this workload or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"kernels_{workload}.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic_record: "):
            rec = json.loads(line[len("traffic_record: "):])
            if rec.get("source_sha256") == sources_sha256(X_KERNEL_SOURCES):
                return rec
    return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def sample_power(torch, step, seconds=4.0):
    """Package power and shader clocks while the step runs back to back for
    `seconds` (untimed, after the timed region): amd-smi is sampled from a
    thread; the cap comes from rocm-smi.  None where the tools are missing or
    print nothing usable."""
    import re
    import shutil
    import subprocess
    import threading

    smi = shutil.which("amd-smi")
    if not smi:
        return None
    samples, stop = [], threading.Event()

    def sampler():
        while not stop.is_set():
            try:
                r = subprocess.run([smi, "metric", "--power", "--clock", "-g", "0", "--csv"], capture_output=True,
                                   text=True, timeout=10)
                lines = [l for l in r.stdout.splitlines() if l.strip()]
                head = next((l.split(",") for l in lines if l.startswith("gpu,")), None)
                row = next((l.split(",") for l in reversed(lines) if l[:1].isdigit()), None)
                if head and row and len(row) == len(head):
                    clk = [float(row[i]) for i, h in enumerate(head) if re.fullmatch(r"gfx_\d+_clk", h)]
                    samples.append((float(row[head.index("socket_power")]), sum(clk) / len(clk) if clk else None))
            except (OSError, ValueError, subprocess.SubprocessError):
                pass
            time.sleep(0.05)

    th = threading.Thread(target=sampler, daemon=True)
    th.start()
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds:
        step()
        torch.cuda.synchronize()
        n += 1
    stop.set()
    th.join(timeout=15)
    if len(samples) < 3:
        return None
    # the first samples may predate the load
    pw = [x[0] for x in samples[1:]]
    ck = [x[1] for x in samples[1:] if x[1] is not None]
    cap = None
    rs = shutil.which("rocm-smi")
    if rs:
        try:
            r = subprocess.run([rs, "--showmaxpower"], capture_output=True, text=True, timeout=20)
            m = re.search(r"Max Graphics Package Power \(W\):\s*([0-9.]+)", r.stdout)
            cap = float(m.group(1)) if m else None
        except (OSError, subprocess.SubprocessError):
            cap = None
    return {"socket_power_w_median": float(np.median(pw)), "socket_power_w_max": float(np.max(pw)),
            "power_cap_w": cap, "shader_clock_mhz_median": float(np.median(ck)) if ck else None,
            "samples": len(pw), "steps_run": n, "seconds": seconds,
            "how": "amd-smi metric --power --clock while the step ran back to back, untimed"}


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


def cpu_model() -> str:
    """The first processor's model name, with its family / model / stepping
    numbers (virtual machines often report only a generic name)."""
    fields = {}
    try:
        for line in open("/proc/cpuinfo"):
            if not line.strip():
                break
            k, _, v = line.partition(":")
            fields[k.strip()] = v.strip()
    except OSError:
        pass
    name = fields.get("model name", "unknown")
    ids = [f"{k} {fields[k]}" for k in ("cpu family", "model", "stepping") if k in fields]
    return f"{name} ({', '.join(ids)})" if ids else name


def cpu_baseline(inp, wl, target_s=CPU_BASELINE_TARGET_S):
    """The FP64 oracle on a bounded, deterministic sample of the workload: random
    (bin, pixel) outputs x all segments, X and Gamma.  Median rate of three runs
    on all host threads, plus one run on a single thread."""
    import oracle

    oracle.build()
    tg, fgd = wl.tgrid, wl.fgrid
    npix = 12 * wl.nside ** 2
    gh = inp["gamma"].cpu().numpy()
    th = inp["tau"].cpu().numpy()
    threads = oracle.default_threads()
    rng = np.random.default_rng(77)

    def run(n, nthreads):
        cols = rng.integers(0, fgd.nf, n)
        pix = rng.integers(0, npix, n)
        t0 = time.perf_counter()
        oracle.maps_at(inp["C_host"], inp["w_host"], fgd.f0, fgd.df, fgd.k0, gh, th, cols, pix, nthreads=nthreads)
        return time.perf_counter() - t0

    # calibrate on a run of at least half a second, then size each timed run
    # for a quarter of the target
    n0 = 2000
    dt0 = run(n0, threads)
    while dt0 < 0.5 and n0 < 4e7:
        n0 *= 4
        dt0 = run(n0, threads)
    n = int(max(n0, min(4e7, n0 * 0.25 * target_s / max(dt0, 1e-3))))
    dts = [run(n, threads) for _ in range(3)]
    dt = float(np.median(dts))
    n1 = int(max(200, n / max(threads, 1)))
    dt1 = run(n1, 1)
    return {"value": n * tg.nt / dt, "unit": "terms/s", "cores": threads, "kind": "oracle",
            "single_core_value": n1 * tg.nt / dt1, "cpu_model": cpu_model(),
            "runs_s": [round(x, 3) for x in dts],
            "sample": f"{n} random (bin, pixel) outputs x all {tg.nt} segments (X and Gamma) per run, "
                      f"median of 3 runs on {threads} threads ({dt:.1f} s); single thread: {n1} outputs in {dt1:.1f} s"}


def result_errors(sg, torch, inp, wl, X, G, Xbb, Gbb):
    """Errors of the step's outputs against the FP64 oracle on the same stored
    inputs, on a deterministic sample: 4 full rows (bins) and 3 full columns
    (pixels).  X: max |dX| / S (S = sum_t |w gamma| |C|), the row-wise
    ||dX||_inf / ||X_ref||_inf over the full rows, and the elementwise relative
    error where |X_ref| >= 0.1 S; Gamma: elementwise relative; the broadband maps
    at the full columns (Xbb against sum_k S, Gbb relative)."""
    import oracle

    oracle.build()
    fgd = wl.fgrid
    npix = 12 * wl.nside ** 2
    rows, cols = synth.random_selection(40 + 3, fgd.nf, npix, 4, 3)
    ri, ci = torch.from_numpy(rows).to(X.device), torch.from_numpy(cols).to(X.device)
    Xs = X[ri, ci].double().cpu().numpy()
    Gs = G[ri, ci].double().cpu().numpy()
    gh, th = inp["gamma"].cpu().numpy(), inp["tau"].cpu().numpy()
    Xo, Go, S = oracle.maps_at(inp["C_host"], inp["w_host"], fgd.f0, fgd.df, fgd.k0, gh, th, rows, cols)
    dX = np.abs(Xs - Xo)
    out = {"x_max_abs_over_S": float(np.max(dX / S)), "gamma_max_rel": float(np.max(np.abs(Gs - Go) / Go))}
    nrow = np.unique(rows[:4 * npix]).size
    rw = [float(np.max(dX[i * npix:(i + 1) * npix]) / np.max(np.abs(Xo[i * npix:(i + 1) * npix])))
          for i in range(nrow)]
    out["x_rowwise_inf_rel"] = max(rw)
    big = np.abs(Xo) >= 0.1 * S
    out["x_elementwise_rel_where_ge_0.1S"] = float(np.max(dX[big] / np.abs(Xo[big]))) if big.any() else None
    out["x_elements_ge_0.1S"] = int(big.sum())
    # broadband maps at the full columns (all bins of 3 pixels)
    c0 = 4 * npix
    H = synth.spectrum_H(fgd.freqs())
    pcols = np.unique(cols[c0:])
    xb, gb, xbe, gbe = [], [], [], []
    for p in pcols:
        m = cols[c0:] == p
        k = rows[c0:][m]
        xo, go, so = Xo[c0:][m], Go[c0:][m], S[c0:][m]
        order = np.argsort(k)
        xbo, gbo, sbo = xo[order].sum(), (H[k[order]] * go[order]).sum(), so[order].sum()
        xbe.append(abs(float(Xbb[int(p)]) - xbo) / sbo)
        gbe.append(abs(float(Gbb[int(p)]) - gbo) / gbo)
    out["xbb_max_abs_over_sumS"] = float(max(xbe))
    out["gbb_max_rel"] = float(max(gbe))
    out["sample"] = f"{nrow} full bins x {npix} pixels + {pcols.size} full pixels x {fgd.nf} bins ({rows.size} outputs)"
    return out


def batched_measure(torch, sg, steps):
    """Batched form (three baselines with uneven jobs: AB nside 64 full band, AC
    nside 32 20-500 Hz, BC nside 16 100-300 Hz) as one autotuned plan replayed
    from a HIP graph, against the plain path (one make_maps_band call per job),
    same box, same inputs; the outputs of the two are compared bit for bit."""
    dev = torch.device("cuda:0")
    jobs, terms = [], 0
    for wl in synth.batched_jobs():
        tg, fgd = wl.tgrid, wl.fgrid
        npix = 12 * wl.nside ** 2
        gamma, tau = sg.build_geometry(synth.baseline_sites(wl.baseline), wl.nside,
                                       sg.TGrid(tg.nt, tg.t0, tg.stride, tg.dur), device=dev)
        f = fgd.freqs()
        C = synth.noise_csd(wl.noise_seed, tg.nt, f, dtype=np.complex64)
        w = synth.weights(f, synth.segment_scale(tg.nt, wl.nonstationary_seed)).astype(np.float32)
        Cd = torch.from_numpy(C).to(dev)
        wd = torch.from_numpy(w).to(dev)
        Hd = torch.from_numpy(synth.spectrum_H(f).astype(np.float32)).to(dev)
        X = torch.empty((fgd.nf, npix), device=dev)
        G = torch.empty_like(X)
        Xbb = torch.empty(npix, device=dev)
        Gbb = torch.empty_like(Xbb)
        jobs.append(sg.Job(Cd, wd, sg.FGrid(fgd.f0, fgd.df), fgd.k0, gamma, tau, X=X, G=G, H=Hd,
                           band=(0, fgd.nf), Xbb=Xbb, Gbb=Gbb))
        terms += tg.nt * fgd.nf * npix
        log(f"job {wl.name}: nside {wl.nside} nf {fgd.nf} k0 {fgd.k0}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = sg.Plan(jobs, autotune=True)
    log(f"plan created in {time.perf_counter() - t0:.1f} s: {plan.describe()}")
    ws = [torch.empty(sg.band_maps_workspace_bytes(j.w.shape[0], j.w.shape[1], j.gamma.shape[1], True),
                      dtype=torch.uint8, device=dev) for j in jobs]

    def plain():
        for j, wsp in zip(jobs, ws):
            sg.make_maps_band(j.C, j.w, j.fgrid, j.k0, j.gamma, j.tau, j.H, *j.band, out=(j.X, j.G, j.Xbb, j.Gbb),
                              workspace=wsp)

    def timed(fn, k):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    ms_plan = timed(plan.launch, steps)
    log(f"plan: {ms_plan:.2f} ms per launch")
    ms_plain = timed(plain, steps)
    log(f"plain path: {ms_plain:.2f} ms per pass")
    # the plain path's outputs (last) against one more plan replay
    ref = [[t.clone() for t in (j.X, j.G, j.Xbb, j.Gbb)] for j in jobs]
    plan.launch()
    torch.cuda.synchronize()
    equal = all(torch.equal(t, r) for j, rr in zip(jobs, ref) for t, r in zip((j.X, j.G, j.Xbb, j.Gbb), rr))
    out = {"workload": "batched_AB64_AC32_BC16", "terms_per_step": terms, "jobs": len(jobs),
           "plan": {"value": terms / (ms_plan * 1e-3), "ms_per_step": ms_plan},
           "plain_path": {"value": terms / (ms_plain * 1e-3), "ms_per_step": ms_plain},
           "outputs_bitwise_equal": bool(equal), "schedule": plan.describe()}
    plan.close()
    del jobs, ws, ref
    torch.cuda.empty_cache()
    return out


def bench_batched(args, torch, sg):
    """Batched form alone (see batched_measure)."""
    r = batched_measure(torch, sg, args.steps)
    out = {
        "metric": "map terms/s (t*f*pix) for X+Gamma", "value": r["plan"]["value"], "unit": "terms/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": r["plan"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE_LABEL, "data": "synthetic",
        "config": {"workload": r["workload"], "terms_per_step": r["terms_per_step"], "jobs": r["jobs"],
                   "parallelism": "single GPU"},
        "plain_path": r["plain_path"], "outputs_bitwise_equal": r["outputs_bitwise_equal"], "plan": r["schedule"],
    }
    print(json.dumps(out), flush=True)


def bench_fisher_overlap(args, torch, sg):
    """Overlap-corrected Fisher diagonal (neighbour terms of 50%-overlapping
    windows) over the full band of one workload, against the plain diagonal."""
    dev = torch.device("cuda:0")
    wl = synth.workload(args.workload)
    tg, fgd = wl.tgrid, wl.fgrid
    npix = 12 * wl.nside ** 2
    f = fgd.freqs()
    g, t = sg.build_geometry(synth.baseline_sites(wl.baseline), wl.nside,
                             sg.TGrid(tg.nt, tg.t0, tg.stride, tg.dur), device=dev)
    v = synth.weights(f, synth.segment_scale(tg.nt, 7))
    u, w = synth.overlap_series(v)
    vd, ud, wd = (torch.from_numpy(a.astype(np.float32)).to(dev) for a in (v, u, w))
    del v, u, w
    G = torch.empty((fgd.nf, npix), dtype=torch.float32, device=dev)
    ws = torch.empty(sg.fisher_overlap_workspace_bytes(tg.nt, fgd.nf, npix), dtype=torch.uint8, device=dev)
    fg = sg.FGrid(fgd.f0, fgd.df)
    C0 = torch.zeros((tg.nt, fgd.nf), dtype=torch.complex64, device=dev)
    mws = sg.make_workspace(tg.nt, fgd.nf, npix, True, device=dev)

    def timed(fn, k):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    t_ov = timed(lambda: sg.fisher_overlap(vd, ud, wd, fg, fgd.k0, g, t, out=G, workspace=ws), args.steps)
    t_plain = timed(lambda: sg.make_maps(C0, vd, fg, fgd.k0, g, t, want_x=False, out=(None, G), workspace=mws),
                    args.steps)
    terms = tg.nt * fgd.nf * npix
    log(f"overlap-corrected Fisher diagonal: {t_ov:.2f} ms; plain diagonal {t_plain:.2f} ms")
    print(json.dumps({"metric": "overlap-corrected Fisher diagonal terms/s (t*f*pix)", "value": terms / (t_ov * 1e-3),
                      "unit": "terms/s", "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": t_ov,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE_LABEL,
                      "data": "synthetic", "config": {"workload": wl.name + "_fisher_overlap", "nt": tg.nt,
                                                      "nf": fgd.nf, "npix": npix, "parallelism": "single GPU"},
                      "plain_diagonal_ms": t_plain}), flush=True)


PEAK_LDS_TBPS = 256 * 128 * 2.4e9 / 1e12  # 256 CUs x 128 B/clk of LDS reads x 2.4 GHz
FISHER_TABLE_BYTES_PER_TERM = 16          # one float4 cubic per (t, p, q) term


def bench_fisher_full(args, torch, sg):
    """Full Fisher matrix of the whole band (Eq. eq_fisher) and --cg-iters
    conjugate-gradient steps towards the clean map, for one folded day of
    --workload; the dirty map comes from make_maps + reduce_band (untimed).
    --fisher-weights separable: w = a(t) b(f) (one delay table); general: the
    non-stationary weights of synth.nonstationary_weights (full rank, one table
    per segment, sgwb_fisher_full_general)."""
    dev = torch.device("cuda:0")
    wl = synth.workload(args.workload)
    tg, fgd = wl.tgrid, wl.fgrid
    npix = 12 * wl.nside ** 2
    inp = make_inputs(sg, torch, wl, dev)
    f = fgd.freqs()
    a = torch.from_numpy(synth.segment_scale(tg.nt, wl.nonstationary_seed).astype(np.float32)).to(dev)
    b = torch.from_numpy((synth.spectrum_H(f) / synth.noise_psd(f) ** 2).astype(np.float32)).to(dev)
    fg = sg.FGrid(fgd.f0, fgd.df)
    X, Gk = sg.make_maps(inp["C"], inp["w"], fg, fgd.k0, inp["gamma"], inp["tau"], antipodal=True)
    Xbb, _ = sg.reduce_band(X, Gk, inp["H"], 0, fgd.nf)
    del X, Gk
    G = torch.empty((npix, npix), dtype=torch.float32, device=dev)
    P = torch.empty(npix, dtype=torch.float32, device=dev)
    general = args.fisher_weights == "general"
    if general:
        del a, b
        wg = torch.from_numpy(synth.nonstationary_weights(f, tg.nt, wl.nonstationary_seed or 1)
                              .astype(np.float32)).to(dev)
        ws = torch.empty(sg.fisher_full_general_workspace_bytes(fg, fgd.k0, 0, fgd.nf, tg.nt, npix,
                                                                not args.fisher_plain),
                         dtype=torch.uint8, device=dev)

        def full():
            sg.fisher_full_general(wg, inp["H"], fg, fgd.k0, 0, fgd.nf, inp["gamma"], inp["tau"], out=G,
                                   workspace=ws, antipodal=not args.fisher_plain)
    else:
        ws = torch.empty(sg.fisher_full_workspace_bytes(fg, fgd.k0, fgd.nf, tg.nt, npix), dtype=torch.uint8,
                         device=dev)

        def full():
            sg.fisher_full(a, b, inp["H"], fg, fgd.k0, 0, fgd.nf, inp["gamma"], inp["tau"], out=G, workspace=ws,
                           antipodal=not args.fisher_plain)

    def clean():
        sg.clean_map_cg(G, Xbb, args.cg_iters, out=P)

    def timed(fn, k):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    t_full = timed(full, args.steps)
    t_cg = timed(clean, args.steps)
    resid = float(torch.linalg.norm(G.double() @ P.double() - Xbb.double()) / torch.linalg.norm(Xbb.double()))
    terms = tg.nt * npix * (npix + 1) // 2
    # table lookups actually made: the whole upper triangle, or with antipodal
    # seeds the two northern blocks' triangles (about half)
    nh = npix // 2
    lookups = tg.nt * (nh * (nh + 1) if not args.fisher_plain else npix * (npix + 1) // 2)
    tbps = lookups * FISHER_TABLE_BYTES_PER_TERM / (t_full * 1e-3) / 1e12
    log(f"full Fisher matrix {npix}^2 over {tg.nt} segments: {t_full:.2f} ms; CG x{args.cg_iters}: {t_cg:.2f} ms; "
        f"relative residual {resid:.3e}")
    print(json.dumps({"metric": "full Fisher matrix pair-terms/s (t*p*q, q>=p)", "value": terms / (t_full * 1e-3),
                      "unit": "terms/s", "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": t_full,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                      "dtype": "f32 table lookups, f64 delay table" + ("s (f64 MFMA)" if general else ""),
                      "data": "synthetic", "config": {"workload": wl.name + "_fisher_full", "nt": tg.nt,
                                                      "nf": fgd.nf, "npix": npix, "parallelism": "single GPU",
                                                      "antipodal_blocks": not args.fisher_plain,
                                                      "weights": args.fisher_weights,
                                                      "workspace_bytes": int(ws.numel()),
                                                      "table_lookups": lookups},
                      "roofline": {"bound": "lds", "achieved": tbps * 1e3, "peak": PEAK_LDS_TBPS * 1e3,
                                   "unit": "GB/s", "frac": tbps / PEAK_LDS_TBPS, "traffic": None},
                      "clean_map": {"cg_iters": args.cg_iters, "ms": t_cg, "relative_residual": resid}}),
          flush=True)


PEAK_HBM_TBPS = 8.0  # MI355X HBM3E


def bench_network(args, torch, sg):
    """Network sum over the three baselines AB, AC, BC (the sum over I of
    Eq. eq:narrowband) of their narrowband dirty maps, then the isotropic and a
    directed contraction (Sec. V) of the summed map, for --workload.  The maps
    are the library's own dirty maps of each baseline's synthetic data."""
    dev = torch.device("cuda:0")
    maps = []
    for i, bl in enumerate(("AB", "AC", "BC")):
        wl = synth.workload(args.workload, baseline=bl)
        wl.noise_seed += i  # each baseline its own noise
        tg, fgd = wl.tgrid, wl.fgrid
        npix = 12 * wl.nside ** 2
        inp = make_inputs(sg, torch, wl, dev)
        X, _ = sg.make_maps(inp["C"], inp["w"], sg.FGrid(fgd.f0, fgd.df), fgd.k0, inp["gamma"], inp["tau"],
                            want_gamma=False)
        maps.append(X)
        del inp
        torch.cuda.empty_cache()
        log(f"dirty map of {bl} ready")
    nf = maps[0].shape[0]
    out = torch.empty_like(maps[0])
    # a directed search's pixel set: the pixels within 5 degrees of a direction
    c, _ = sg.healpix_centres(wl.nside, device=dev)
    d = torch.tensor([0.3, -0.5, 0.81], dtype=torch.float64, device=dev)
    pix = torch.nonzero((c @ (d / d.norm())) >= np.cos(np.radians(5.0))).flatten().to(torch.int32)
    iso = torch.empty(nf, dtype=torch.float32, device=dev)
    dire = torch.empty(nf, dtype=torch.float32, device=dev)

    def timed(fn, k):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    t_sum = timed(lambda: sg.network_sum(maps, out=out), args.steps)
    t_iso = timed(lambda: sg.contract_pixels(out, None, out=iso), args.steps)
    t_dir = timed(lambda: sg.contract_pixels(out, pix, out=dire), args.steps)
    n = out.numel()
    sum_bytes = (len(maps) + 1) * n * 4
    gbps = sum_bytes / (t_sum * 1e-3) / 1e9
    log(f"network sum of {len(maps)} maps ({n} values each): {t_sum:.3f} ms, {gbps:.0f} GB/s; isotropic contraction "
        f"{t_iso:.3f} ms; directed contraction over {pix.numel()} pixels {t_dir:.3f} ms")
    print(json.dumps({"metric": "network sum GB/s (HBM bytes read + written)", "value": gbps, "unit": "GB/s",
                      "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": t_sum, "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None, "dtype": "f32 maps, f64 sums", "data": "synthetic",
                      "config": {"workload": wl.name + "_network_sum", "baselines": 3, "nf": nf,
                                 "npix": int(out.shape[1]), "parallelism": "single GPU"},
                      "roofline": {"bound": "hbm", "achieved": gbps, "peak": PEAK_HBM_TBPS * 1e3, "unit": "GB/s",
                                   "frac": gbps / (PEAK_HBM_TBPS * 1e3), "traffic": None},
                      "isotropic_contraction": {"ms": t_iso, "GBps": n * 4 / (t_iso * 1e-3) / 1e9},
                      "directed_contraction": {"ms": t_dir, "pixels": int(pix.numel())}}), flush=True)


def bench_broadband(args, torch, sg):
    """The served form's largest query alone: the broadband maps of a full day,
    nside 128, 4096 bins of 1/32 Hz (baseline AB), through sgwb_broadband_maps on
    each route: the strip sums of the matrix-core dirty map, and the band summed
    first through per-segment delay tables (the route the cost rule picks)."""
    dev = torch.device("cuda:0")
    tg = synth.TGRID_FULL
    nside, nb, k0 = 128, 4096, 0
    npix = 12 * nside * nside
    fgd = synth.FGRID_FULL
    f = fgd.freqs()[k0:k0 + nb]
    C = synth.noise_csd(31, tg.nt, f, dtype=np.complex64)
    w = synth.weights(f, synth.segment_scale(tg.nt, 7)).astype(np.float32)
    Cd, wd = torch.from_numpy(C).to(dev), torch.from_numpy(w).to(dev)
    H = torch.from_numpy(synth.spectrum_H(f).astype(np.float32)).to(dev)
    sites = synth.baseline_sites("AB")
    g, t = sg.build_geometry(sites, nside, sg.TGrid(tg.nt, tg.t0, tg.stride, tg.dur), device=dev)
    fg = sg.FGrid(fgd.f0, fgd.df)
    tb = sg.baseline_delay_bound(sites)
    res = {}
    for route in ("strips", "table", "auto"):
        ws = torch.empty(max(sg.broadband_maps_workspace_bytes(tg.nt, nb, npix, fg, 0, nb, tb, route=route), 256),
                         dtype=torch.uint8, device=dev)
        Xbb = torch.empty(npix, dtype=torch.float32, device=dev)
        Gbb = torch.empty(npix, dtype=torch.float32, device=dev)

        def call():
            sg.broadband_maps(Cd, wd, fg, k0, g, t, H, 0, nb, tau_bound=tb, route=route, out=(Xbb, Gbb),
                              workspace=ws)

        for _ in range(args.warmup):
            call()
        torch.cuda.synchronize()
        form = sg.last_x_form()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            call()
        e1.record()
        torch.cuda.synchronize()
        res[route] = {"ms": e0.elapsed_time(e1) / args.steps, "form": form}
        log(f"broadband query, route {route} ({form}): {res[route]['ms']:.3f} ms")
        del ws
    ms = res["auto"]["ms"]
    terms = tg.nt * nb * npix
    seed_bytes = tg.nt * npix * 12  # gamma (4 B) and tau (8 B) read once per (segment, pixel)
    print(json.dumps({"metric": "broadband query latency (ms)", "value": ms, "unit": "ms", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": False,
                      "scaling": "weak", "vs_baseline": None, "dtype": "f64 tables and sums, f32 interpolation",
                      "data": "synthetic",
                      "config": {"workload": "broadband_query_nside128_4096_bins", "baseline": "AB", "nt": tg.nt,
                                 "nb": nb, "nside": nside, "npix": npix, "parallelism": "single GPU"},
                      "terms_per_s": terms / (ms * 1e-3),
                      "seed_read_GBps_whole_call": seed_bytes / (ms * 1e-3) / 1e9,
                      "routes": res}), flush=True)


def bench_folded(args, torch, sg):
    """Folded pipeline over --days synthetic sidereal days of the full band: fold
    (v, u, w, x), dirty map of x, overlap-corrected Fisher diagonal, band sums."""
    dev = torch.device("cuda:0")
    wl = synth.workload(args.workload)
    tg, fgd = wl.tgrid, wl.fgrid
    npix = 12 * wl.nside ** 2
    nd, nt, nf = args.days, tg.nt, fgd.nf
    f = torch.from_numpy(fgd.freqs()).to(dev)
    gen = torch.Generator(device=dev).manual_seed(17)
    # per-day inverse variances a_d H / P^2 and circular complex noise of variance P^2
    P = (f / 100.0) ** -2 + 1.0 + (f / 500.0) ** 2
    Hf = (f / 100.0) ** -3
    a_d = torch.rand((nd, nt, 1), generator=gen, device=dev, dtype=torch.float64) + 0.5
    sinv = (a_d * (Hf / P ** 2)).to(torch.float32)
    C = torch.complex(torch.randn((nd, nt, nf), generator=gen, device=dev),
                      torch.randn((nd, nt, nf), generator=gen, device=dev)) * (P / 2 ** 0.5).to(torch.float32)
    present = torch.rand((nd, nt), generator=gen, device=dev) >= 0.02
    g, t = sg.build_geometry(synth.baseline_sites(wl.baseline), wl.nside,
                             sg.TGrid(tg.nt, tg.t0, tg.stride, tg.dur), device=dev)
    fg = sg.FGrid(fgd.f0, fgd.df)
    ones = torch.ones((nt, nf), dtype=torch.float32, device=dev)
    Hs = Hf.to(torch.float32)
    X = torch.empty((nf, npix), dtype=torch.float32, device=dev)
    G = torch.empty_like(X)
    Xbb = torch.empty(npix, dtype=torch.float32, device=dev)
    Gbb = torch.empty_like(Xbb)
    mws = sg.make_workspace(nt, nf, npix, True, device=dev)
    fws = torch.empty(sg.fisher_overlap_workspace_bytes(nt, nf, npix), dtype=torch.uint8, device=dev)
    folded = [torch.empty((nt, nf), dtype=torch.float32, device=dev) for _ in range(3)]
    folded.append(torch.empty((nt, nf), dtype=torch.complex64, device=dev))

    def step(evs=None):
        if evs:
            evs[0].record()
        v, u, w, x = sg.fold(C, sinv, present, synth.HANN_OVERLAP_W, out=folded)
        if evs:
            evs[1].record()
        sg.make_maps(x, ones, fg, fgd.k0, g, t, want_gamma=False, out=(X, None), workspace=mws)
        if evs:
            evs[2].record()
        sg.fisher_overlap(v, u, w, fg, fgd.k0, g, t, out=G, workspace=fws)
        if evs:
            evs[3].record()
        sg.reduce_band(X, G, Hs, 0, nf, out=(Xbb, Gbb))
        if evs:
            evs[4].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    ph = {name: float(np.mean([e[i].elapsed_time(e[i + 1]) for e in evs]))
          for i, name in enumerate(("fold", "dirty_map", "fisher_overlap", "band"))}
    in_bytes = nd * nt * nf * 12 + nd * nt
    terms = nt * nf * npix
    log(f"folded pipeline, {nd} days: {ms:.2f} ms per step, phases {ph}")
    print(json.dumps({"metric": "folded-pipeline map terms/s (t*f*pix, X + overlap-corrected Gamma)",
                      "value": terms / (ms * 1e-3), "unit": "terms/s", "n_gpus": 1, "steps": args.steps,
                      "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
                      "vs_baseline": None, "dtype": DTYPE_LABEL, "data": "synthetic",
                      "config": {"workload": f"{wl.name}_folded_{nd}_days", "days": nd, "nt": nt, "nf": nf,
                                 "npix": npix, "parallelism": "single GPU"},
                      "phases_ms": ph, "fold_GBps": in_bytes / (ph["fold"] * 1e-3) / 1e9}), flush=True)


def serving_sweep(args, torch, sg, rates, duration):
    """Poisson streams of map queries (200 queries/s x 60 s is the served
    workload; other rates for a sweep) against three resident baselines, through
    the continuous-batching server and through the plain per-query path (one
    query at a time, synchronous), same queries, same accuracy (the same
    kernels: each served result is bitwise the direct call's).  Both compute a
    query's broadband maps alone (no narrowband map is written)."""
    dev = torch.device("cuda:0")
    datasets = []
    for i, bl in enumerate(("AB", "AC", "BC")):
        tg, fgd = synth.TGRID_FULL, synth.FGRID_FULL
        f = fgd.freqs()
        C = synth.noise_csd(4 + i, tg.nt, f, dtype=np.complex64)
        w = synth.weights(f, np.ones(tg.nt)).astype(np.float32)
        datasets.append(sg.Dataset(torch.from_numpy(C).to(dev), torch.from_numpy(w).to(dev),
                                   torch.from_numpy(synth.spectrum_H(f).astype(np.float32)).to(dev),
                                   sg.FGrid(fgd.f0, fgd.df), fgd.k0, synth.baseline_sites(bl),
                                   sg.TGrid(tg.nt, tg.t0, tg.stride, tg.dur)))
        del C, w
        log(f"dataset {bl} resident")
    nt = synth.TGRID_FULL.nt
    srv = sg.Server(datasets, slots=args.slots, hbm_budget_bytes=args.arena_gib << 30)
    # build every (baseline, nside) seed matrix once, as a long-running server would have
    warm = [srv.submit(d, n, 0, 1) for d in range(3) for n in synth.NSIDES_SERVED]
    while any(srv.poll(t) is None for t in warm):
        time.sleep(0.001)
    for t in warm:
        srv.release(t)
    geoms = {}
    bounds = [sg.baseline_delay_bound(d.sites) for d in datasets]

    def plain_query(ds, nside, lo, hi):
        d = datasets[ds]
        if (ds, nside) not in geoms:
            geoms[(ds, nside)] = sg.build_geometry(d.sites, nside, d.tgrid, device=dev)
        g, t = geoms[(ds, nside)]
        # the broadband maps alone, as the server computes them (the same route for the same query)
        sg.broadband_maps(d.C[:, lo:hi], d.w[:, lo:hi], d.fgrid, d.k0 + lo, g, t, d.H[lo:hi].contiguous(), 0, hi - lo,
                          tau_bound=bounds[ds])
        torch.cuda.synchronize()

    for ds in range(3):  # warm the plain path's seeds too
        for n in synth.NSIDES_SERVED:
            plain_query(ds, n, 0, 1)

    results = []
    for rate in rates:
        qs = synth.serving_queries(rate, duration)
        terms = sum(nt * (hi - lo) * 12 * n * n for _, _, n, lo, hi in qs)
        # server
        t0 = time.perf_counter()
        tickets = {}
        lag = {}  # ticket -> submission time minus arrival time, s (the loop submits up to a poll late)
        i = 0
        done = {}
        next_log = 10.0
        while len(done) < len(qs):
            now = time.perf_counter() - t0
            while i < len(qs) and qs[i][0] <= now:
                tk = srv.submit(*qs[i][1:])
                if tk < 0:
                    break
                lag[tk] = (time.perf_counter() - t0) - qs[i][0]
                tickets[tk] = i
                i += 1
            for tk in list(tickets):
                r = srv.poll(tk)
                if r is not None:
                    done[tk] = r
                    srv.release(tk)
                    del tickets[tk]
            if now >= next_log:
                log(f"rate {rate}/s server: {now:.0f} s, {len(done)}/{len(qs)} queries done")
                next_log += 10.0
            # sleep until the next arrival, at most 0.1 ms (results are polled meanwhile)
            wait = (qs[i][0] - (time.perf_counter() - t0)) if i < len(qs) else 1e-4
            if wait > 0:
                time.sleep(min(wait, 1e-4))
        assert all(r["status"] == 0 for r in done.values()), "a served query failed"
        # from arrival, as the plain path's: the server's own submit-to-done time plus the submission lag
        lat = np.array([r["t_done"] - r["t_submit"] + lag[tk] for tk, r in done.items()]) * 1e3
        span = max(r["t_done"] for r in done.values()) - min(r["t_submit"] for r in done.values())
        st = srv.stats()
        log(f"rate {rate}/s server: {len(qs)} queries, p50 {np.percentile(lat, 50):.1f} ms, "
            f"p99 {np.percentile(lat, 99):.1f} ms, {terms / span:.3e} terms/s")
        # plain per-query path, same arrivals, first come first served
        t0 = time.perf_counter()
        plat = []
        next_log = 10.0
        for (ta, ds, n, lo, hi) in qs:
            now = time.perf_counter() - t0
            if now < ta:
                time.sleep(ta - now)
            plain_query(ds, n, lo, hi)
            plat.append((time.perf_counter() - t0 - ta) * 1e3)
            if now >= next_log:
                log(f"rate {rate}/s plain: {now:.0f} s, {len(plat)}/{len(qs)} queries done")
                next_log += 10.0
        pspan = time.perf_counter() - t0 - qs[0][0]
        plat = np.array(plat)
        log(f"rate {rate}/s plain: p50 {np.percentile(plat, 50):.1f} ms, p99 {np.percentile(plat, 99):.1f} ms, "
            f"{terms / pspan:.3e} terms/s")
        results.append({"rate_hz": rate, "duration_s": duration, "queries": len(qs), "terms": terms,
                        "server": {"terms_per_s": terms / span, "p50_ms": float(np.percentile(lat, 50)),
                                   "p99_ms": float(np.percentile(lat, 99)), "arena_peak_bytes": st["arena_peak"]},
                        "plain": {"terms_per_s": terms / pspan, "p50_ms": float(np.percentile(plat, 50)),
                                  "p99_ms": float(np.percentile(plat, 99))}})
    srv.close()
    del datasets, geoms
    torch.cuda.empty_cache()
    return results


def bench_serve(args, torch, sg):
    """Serving form alone: a rate sweep (--rates, --duration s each)."""
    results = serving_sweep(args, torch, sg, args.rates, args.duration)
    top = results[-1]
    out = {
        "metric": "map terms/s (t*f*pix) for X+Gamma; p50/p99 query latency", "value": top["server"]["terms_per_s"],
        "unit": "terms/s", "n_gpus": 1, "steps": len(results), "warmup": 1, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE_LABEL, "data": "synthetic",
        "config": {"workload": "serving_poisson", "duration_s": args.duration, "slots": args.slots,
                   "nsides": list(synth.NSIDES_SERVED), "max_band": 4096, "parallelism": "single GPU"},
        "latency_ms": {"p50": top["server"]["p50_ms"], "p99": top["server"]["p99_ms"]},
        "sweep": results,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=3, help="3: full band nside 64 (default); 2: full band nside 32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-errors", action="store_true", help="skip the per-result errors against the oracle")
    ap.add_argument("--no-power", action="store_true", help="skip the untimed package-power sample")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="serving leg of the default run: Poisson queries at 200/s for this long (0: none)")
    ap.add_argument("--batched", action="store_true", help="batched plan of three uneven baseline jobs")
    ap.add_argument("--no-batched-leg", action="store_true", help="leave the batched form out of the default run")
    ap.add_argument("--serve", action="store_true", help="Poisson query stream through the server (rate sweep)")
    ap.add_argument("--folded", action="store_true",
                    help="fold --days synthetic days, then X, overlap-corrected Gamma and band sums")
    ap.add_argument("--days", type=int, default=10)
    ap.add_argument("--fisher-overlap", action="store_true",
                    help="overlap-corrected Fisher diagonal over the full band of --workload")
    ap.add_argument("--broadband", action="store_true",
                    help="the served form's largest query (nside 128, 4096 bins) on both broadband routes")
    ap.add_argument("--network", action="store_true",
                    help="network sum of three baselines' narrowband maps and the contractions, for --workload")
    ap.add_argument("--fisher-full", action="store_true",
                    help="full Fisher matrix of the whole band and the CG clean map for --workload")
    ap.add_argument("--cg-iters", type=int, default=50)
    ap.add_argument("--fisher-weights", choices=["separable", "general"], default="separable",
                    help="full Fisher matrix weights: a(t) b(f), or general non-stationary w(t,f)")
    ap.add_argument("--fisher-plain", action="store_true",
                    help="full Fisher matrix without the antipodal block decomposition")
    ap.add_argument("--rates", type=float, nargs="+", default=[25.0, 50.0, 100.0, 200.0])
    ap.add_argument("--duration", type=float, default=5.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--arena-gib", type=int, default=64)
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
    if args.batched:
        bench_batched(args, torch, sg)
        return
    if args.serve:
        bench_serve(args, torch, sg)
        return
    if args.fisher_overlap:
        bench_fisher_overlap(args, torch, sg)
        return
    if args.folded:
        bench_folded(args, torch, sg)
        return
    if args.fisher_full:
        bench_fisher_full(args, torch, sg)
        return
    if args.broadband:
        bench_broadband(args, torch, sg)
        return
    if args.network:
        bench_network(args, torch, sg)
        return
    wl = synth.workload(args.workload)
    tg, fgd = wl.tgrid, wl.fgrid
    npix = 12 * wl.nside ** 2
    log(f"workload {wl.name}: nt={tg.nt} nf={fgd.nf} npix={npix}")
    inp = make_inputs(sg, torch, wl, dev)
    X = torch.empty((fgd.nf, npix), dtype=torch.float32, device=dev)
    G = torch.empty_like(X)
    Xbb = torch.empty(npix, dtype=torch.float32, device=dev)
    Gbb = torch.empty_like(Xbb)
    ws = torch.empty(sg.band_maps_workspace_bytes(tg.nt, fgd.nf, npix, True), dtype=torch.uint8, device=dev)
    fg = sg.FGrid(fgd.f0, fgd.df)

    # One step: the dirty map with its band sum, then the beam with its band sum
    # (make_maps_band: the map kernels add their tiles' band sums, one small
    # kernel per map adds those up).  Events are recorded on torch's current
    # stream, the stream the library's kernels are queued on.
    def step(evs=None):
        if evs:
            evs[0].record()
        sg.make_maps_band(inp["C"], inp["w"], fg, fgd.k0, inp["gamma"], inp["tau"], None, 0, fgd.nf,
                          want_gamma=False, out=(X, None, Xbb, None), workspace=ws)
        if evs:
            evs[1].record()
        sg.make_maps_band(inp["C"], inp["w"], fg, fgd.k0, inp["gamma"], inp["tau"], inp["H"], 0, fgd.nf,
                          want_x=False, out=(None, G, None, Gbb), workspace=ws)
        if evs:
            evs[2].record()

    # the dirty map's form (read back right after an X call)
    sg.make_maps_band(inp["C"], inp["w"], fg, fgd.k0, inp["gamma"], inp["tau"], None, 0, fgd.nf,
                      want_gamma=False, out=(X, None, Xbb, None), workspace=ws)
    x_form = sg.last_x_form()
    log(f"dirty-map form: {x_form}")
    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {wall:.3f} s")
    t_x = np.array([e[0].elapsed_time(e[1]) for e in evs])
    t_g = np.array([e[1].elapsed_time(e[2]) for e in evs])
    t_step = np.array([e[0].elapsed_time(e[2]) for e in evs])
    ms_per_step = wall * 1e3 / args.steps
    terms = tg.nt * fgd.nf * npix
    x_tflops = X_FLOPS_PER_TERM * terms / (t_x.mean() * 1e-3) / 1e12
    if x_form and x_form.startswith("mfma"):
        rec = recorded_traffic(wl.name)
        roofline = {"bound": "mfma", "kernel": "xm_main_kernel (split-f16 MFMA dirty map)", "achieved": x_tflops,
                    "peak": PEAK_F16_MFMA_TFLOPS, "unit": "TFLOP/s", "frac": x_tflops / PEAK_F16_MFMA_TFLOPS,
                    "traffic": rec["hbm_bytes"] if rec else None, "flops_per_term": X_FLOPS_PER_TERM,
                    "x_form": x_form, "launch_ms": float(t_x.mean()),
                    "issued_flops_per_term": ISSUED_FLOPS_PER_TERM[x_form],
                    "issued_tflops": ISSUED_FLOPS_PER_TERM[x_form] * terms / (t_x.mean() * 1e-3) / 1e12}
        if rec:
            roofline["traffic_algorithmic_bytes"] = rec["algorithmic_bytes"]
    else:
        roofline = {"bound": "alu", "kernel": "dirty_map_kernel<float, pair>", "achieved": x_tflops,
                    "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s", "frac": x_tflops / PEAK_FP32_VECTOR_TFLOPS,
                    "traffic": None, "flops_per_term": X_FLOPS_PER_TERM, "x_form": x_form,
                    "launch_ms": float(t_x.mean())}

    power = None
    if not args.no_power:
        log("package power while the step runs back to back (untimed)")
        power = sample_power(torch, step)
        log(f"power: {power}")

    if args.copy_calib_mib:
        nbytes = args.copy_calib_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {nbytes} bytes read, {nbytes} bytes written")
        del src, dst

    errors = None
    if not args.no_errors:
        log("errors against the FP64 oracle on a sample of the outputs")
        errors = result_errors(sg, torch, inp, wl, X, G, Xbb, Gbb)
        log(f"errors: {errors}")

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on the host cores")
        cpu = cpu_baseline(inp, wl)

    del X, G, ws
    inp.pop("C_host"), inp.pop("w_host")
    torch.cuda.empty_cache()
    batched = None
    if not args.no_batched_leg:
        log("batched leg: three uneven jobs as one plan against one call per job")
        batched = batched_measure(torch, sg, args.steps)

    serving = None
    if args.serve_seconds > 0:
        log(f"serving leg: 200 queries/s for {args.serve_seconds:.0f} s, server and plain path")
        serving = serving_sweep(args, torch, sg, [200.0], args.serve_seconds)[0]

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
        "dtype": DTYPE_LABEL,
        "data": "synthetic (seeded noise model + injected point sources)",
        "config": {"workload": wl.name, "baseline": wl.baseline, "nt": tg.nt, "nf": fgd.nf, "nside": wl.nside,
                   "npix": npix, "f0_hz": fgd.f0, "df_hz": fgd.df, "terms_per_step": terms,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "phases_ms": {"dirty_map": float(t_x.mean()), "beam": float(t_g.mean())},
        "step_latency_ms": {"p50": float(np.percentile(t_step, 50)), "p99": float(np.percentile(t_step, 99))},
        "errors_vs_oracle": errors,
        "cpu_baseline": cpu,
        "power": power,
    }
    if batched:
        out["batched"] = batched
    if serving:
        out["latency_ms"] = {"p50": serving["server"]["p50_ms"], "p99": serving["server"]["p99_ms"],
                             "what": "served query latency, Poisson 200 queries/s"}
        out["serving"] = serving
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
