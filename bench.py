"""Benchmark of the MI355X burst merge.

One step = one forward merge (every stage of the hot path) of the 12 MP x 8
frame burst (4032x3024 RGGB uint16, occluder, scale 1, 16 px tiles), inputs
resident in HBM. Prints one JSON line with input-Bayer MP/s, the dominant
kernel's roofline position and the FP64 oracle's CPU rate on a bounded sample.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-cpu-baseline]
                    [--no-batch] [--no-grad] [--no-stream] [--no-align] [--no-configs]
    python bench.py --only-config {1,3} [--steps K]   (that workload's merge alone)

More legs follow the headline measurement and are reported inside its line:
the low-light workload (15 x 1512 x 2016 at scale 2) and the small 8 x 256 x
256 burst, the same burst merged frame by frame through the streaming calls, its tile
alignment (with its ground-truth error split by tile structure, with and
without the noise gate) and the raw-burst-to-RGB time (alignment then merge), the
64-burst batched workload (one graph replay vs per-burst launches) and the
differentiation workload (16 bursts of 8 x 768 x 1024 at scale 2, forward
plus adjoint).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks and unit counts.
HBM_PEAK_GBS = 8000.0
CUS, CLOCK_GHZ, LANES = 256, 2.4, 64
ALU_PEAK_TOPS = CUS * LANES * CLOCK_GHZ / 1000.0   # vector lane-operations: 39.3 T/s


# Algorithmic vector operations of the method (see the op-count table in the
# design notes): adds, multiplies, fmas, compares/min/max/selects count 1,
# divide / square root / exp count 4 (their issue cost).
OPS_SAMPLE = 161.0      # per output pixel and frame: nine-sample weights and accumulation
OPS_OMEGA = 79.0        # per half-res pixel and frame: luma, structure tensor, eigen, S.1, Omega
OPS_ROBUST = 98.0       # per half-res pixel and aligned frame: guide means, eq. 5-6, 5x5 min
# Adjoint of the accumulation: the recomputed weights (the forward count less its
# accumulation) plus dL/de, dL/drho, the offset moments, dL/dOmega_bar, dL/dp and
# the four corner projections onto the six covariance scalars.
OPS_ADJ_SAMPLE = 337.0  # per output pixel and frame
OPS_ADJ_OMEGA = 99.0    # per half-res pixel and frame: Omega and its ten per-scalar factors


def algorithmic_ops(desc) -> dict:
    """Algorithmic operation count of each kernel for one merge of `desc`."""
    n, hp = desc.n_frames, (desc.height // 2) * (desc.width // 2)
    pf = n * desc.out_height * desc.out_width
    return {"k_merge": OPS_SAMPLE * pf + OPS_OMEGA * n * hp,
            "k_robust": OPS_ROBUST * (n - 1) * hp}


def algorithmic_bytes(desc) -> dict:
    """Each input byte read once, each output byte written once, per kernel."""
    n, h, w = desc.n_frames, desc.height, desc.width
    hp = (h // 2) * (w // 2)
    tiles = desc.tiles_y * desc.tiles_x
    return {"k_merge": 2 * n * h * w + 8 * n * tiles + 4 * (n - 1) * hp
            + 12 * desc.out_height * desc.out_width,
            "k_robust": 2 * n * h * w + 12 * n * tiles + 4 * (n - 1) * hp,
            "total": 2 * n * h * w + 8 * n * tiles + 12 * desc.out_height * desc.out_width}


# Sources whose code the merge kernel's traffic figures depend on.
TRAFFIC_SOURCES = ("paper_1905_03277_amd/csrc/merge.hip", "paper_1905_03277_amd/csrc/merge_tile.h",
                   "paper_1905_03277_amd/csrc/merge_common.h", "paper_1905_03277_amd/csrc/omega.h",
                   "paper_1905_03277_amd/csrc/device_util.h", "paper_1905_03277_amd/csrc/hmfsr_internal.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "merge_fwd_12mp_x8_traffic.md")
CALIB_BYTES = 256 << 20    # the plain copy the HBM counters are scaled by


def source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per k_merge launch from the committed counter summary, or
    None when the kernel sources changed since the counters were taken."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    fields = dict(line.split("=", 1) for line in text.splitlines() if line.startswith(("hash=", "bytes=")))
    if fields.get("hash", "").strip() != source_hash():
        return None
    return int(fields["bytes"])


def calibration_copy(dev):
    """A plain device copy of CALIB_BYTES (read + write), outside any timed
    region: the reference the FETCH_SIZE / WRITE_SIZE counters are scaled by."""
    import torch
    a = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    torch.neg(a, out=b)   # one elementwise kernel: reads and writes CALIB_BYTES
    torch.cuda.synchronize()
    del a, b


def _plain(obj) -> dict:
    """A descriptor or tuning as a plain dict (the oracle reads either)."""
    import dataclasses
    return {f.name: getattr(obj, f.name) for f in dataclasses.fields(obj) if f.name != "noise_table"}


def _oracle_window(job):
    """One oracle merge of an output window (runs in a worker process with one
    thread): returns the input Bayer pixels behind the window."""
    fr, mo, dd, tun, ry, rx, in_px = job
    from threadpoolctl import threadpool_limits
    import oracle.merge as om
    with threadpool_limits(limits=1):
        om.merge_window(fr, mo, dd, tun, ry, rx)
    return in_px


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(burst, single_s: float = 8.0, all_s: float = 25.0, max_workers: int = 16):
    """Time the FP64 oracle on the same burst on this host's cores: one thread
    on windows of 256 x 256 output pixels, then every core (one single-thread
    worker process each, at most ``max_workers``) on row bands of the whole
    image, until the bands run out or the time budget does."""
    import concurrent.futures as cf
    import multiprocessing as mp
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity_util import crop_case

    f, m = burst.numpy()
    d = burst.desc
    dd, tun = _plain(d), _plain(burst.tuning)
    n = d.n_frames

    # single thread, windows spread over the image
    S = 256
    spots = [(d.out_height // 2, d.out_width // 2), (d.out_height // 4, d.out_width // 4),
             (3 * d.out_height // 4, d.out_width // 3)]
    px = 0.0
    t0 = time.perf_counter()
    i = 0
    while time.perf_counter() - t0 < single_s:
        oy, ox = spots[i % len(spots)]
        fr, mo, dc, ry, rx = crop_case(f, m, d, oy, ox, S, S)
        px += _oracle_window((fr, mo, _plain(dc), tun, ry, rx, n * (S / d.scale) ** 2))
        i += 1
    dt1 = time.perf_counter() - t0
    single = px / dt1 / 1e6

    # every core: bands of 192 output rows covering the whole output
    cores = len(os.sched_getaffinity(0))
    workers = max(1, min(cores, max_workers))
    band = 192
    jobs = []
    for oy in range(0, d.out_height, band):
        rows = min(band, d.out_height - oy)
        fr, mo, dc, ry, rx = crop_case(f, m, d, oy, 0, rows, d.out_width)
        jobs.append((fr, mo, _plain(dc), tun, ry, rx, n * rows * d.out_width / d.scale ** 2))
    done_px, done = 0.0, 0
    env_threads = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env_threads:
        os.environ[k] = "1"
    try:
        with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
            list(ex.map(_oracle_window, [jobs[0]] * workers))   # start the workers and their imports
            t0 = time.perf_counter()
            pending = {ex.submit(_oracle_window, j) for j in jobs}
            while pending:
                fin, pending = cf.wait(pending, timeout=max(0.1, all_s - (time.perf_counter() - t0)),
                                       return_when=cf.FIRST_COMPLETED)
                for fu in fin:
                    done_px += fu.result()
                    done += 1
                if time.perf_counter() - t0 >= all_s:
                    for fu in pending:
                        fu.cancel()
                    break
            dt = time.perf_counter() - t0
    finally:
        for k, v in env_threads.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    whole = done == len(jobs)
    return {"value": round(done_px / dt / 1e6, 3), "unit": "MP/s", "cores": workers, "kind": "oracle",
            "sample": (f"{done} of {len(jobs)} bands of {band} output rows x {d.out_width} px (x{n} frames, "
                       f"each with its input halo) of the 12 MP x 8 burst, {dt:.1f} s, {workers} single-thread "
                       f"worker processes" + (" (the whole image)" if whole else "")),
            "host_cores_available": cores, "cpu_model": cpu_model(),
            "single_thread": {"value": round(single, 3), "unit": "MP/s", "cores": 1,
                              "sample": f"{i} windows of {S}x{S} output px (x{n} frames), {dt1:.1f} s"}}


def bench_batch(dev, reps: int = 3) -> dict:
    """The uneven batched workload (64 bursts, 2-15 frames, 0.2-12 MP, scale
    1/1.5/2): one replay of the captured persistent-kernel graph versus one
    hmfsr_merge launch sequence per burst, after autotuning one burst of every
    (scale, frame-count) class present."""
    import torch
    from paper_1905_03277_amd import synth, torch_ops

    print("[bench] generating the 64-burst batch", file=sys.stderr, flush=True)
    bursts = synth.make_batch(64, device=dev)
    args = [(b.frames, b.motion, b.desc, b.tuning) for b in bursts]
    outs = [torch.empty((3, b.desc.out_height, b.desc.out_width), dtype=torch.float32, device=dev)
            for b in bursts]
    tuned = {}
    for (f, m, d, t), o in zip(args, outs):
        key = (0 if d.scale <= 1 else 1 if d.scale <= 1.5 else 2,
               0 if d.n_frames <= 4 else 1 if d.n_frames <= 8 else 2)
        if key not in tuned:
            tuned[key] = torch_ops.autotune(f, m, d, t, out=o)[0]
    torch.cuda.synchronize()
    in_mp = sum(d.n_frames * d.height * d.width for f, m, d, t in args) / 1e6
    stream = torch.cuda.current_stream()

    def timeit(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    print("[bench] batch: graph replay vs per-burst launches", file=sys.stderr, flush=True)
    ms_graph = timeit(lambda: torch_ops.merge_batch(args, outs))
    ms_loop = timeit(lambda: [torch_ops.merge(f, m, d, t, out=o) for (f, m, d, t), o in zip(args, outs)])
    # per-burst rates of the launch loop
    rates = []
    for f, m, d, t in args:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        torch_ops.merge(f, m, d, t)
        e1.record(stream)
        torch.cuda.synchronize()
        rates.append(d.n_frames * d.height * d.width / 1e6 / (e0.elapsed_time(e1) / 1e3))
    rates.sort()
    return {"workload": "64 bursts, frames U{2..15}, sizes {512x384, 1024x768, 2016x1512, "
                        "4032x3024}, scale {1, 1.5, 2}",
            "input_MP": round(in_mp, 1), "ms_graph": round(ms_graph, 3), "ms_per_burst_loop": round(ms_loop, 3),
            "MPs_graph": round(in_mp / (ms_graph / 1e3), 1),
            "MPs_per_burst_loop": round(in_mp / (ms_loop / 1e3), 1),
            "speedup": round(ms_loop / ms_graph, 3),
            "per_burst_MPs_loop": {"min": round(rates[0], 1), "median": round(rates[len(rates) // 2], 1),
                                   "max": round(rates[-1], 1)},
            "tuned_shapes": {f"{k[0]}/{k[1]}": v for k, v in tuned.items()}}


def bench_config(cfg: int, dev, reps: int = 10) -> dict:
    """Forward merge of another workload: config 3 (Super-Res Zoom low light,
    15 x 1512 x 2016 at scale 2, SNR-11 tuning) or config 1 (8 x 256 x 256 at
    scale 1, launch-bound). Whole-merge rate by events, per-kernel times by
    the library's event timing, and k_merge's position on the ALU roofline."""
    import torch
    from paper_1905_03277_amd import binding, synth, torch_ops

    print(f"[bench] config {cfg}", file=sys.stderr, flush=True)
    b = synth.make_config(cfg, device=dev)
    d = b.desc
    out = torch.empty((3, d.out_height, d.out_width), dtype=torch.float32, device=dev)

    def step():
        torch_ops.merge(b.frames, b.motion, d, b.tuning, out=out)

    stream = torch.cuda.current_stream()
    for _ in range(3):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    binding.hmfsr_profile_begin()
    for _ in range(reps):
        step()
    kern = {k: tot / max(cnt, 1) for k, (tot, cnt) in binding.hmfsr_profile_end().items()}
    in_mp = d.n_frames * d.height * d.width / 1e6
    ops = algorithmic_ops(d)["k_merge"]
    ach = ops / (kern["k_merge"] / 1e3) / 1e12
    byts = algorithmic_bytes(d)["total"]
    return {"workload": f"forward merge, {d.n_frames} frames {d.width}x{d.height} RGGB, scale {d.scale:g}, "
                        f"{d.tile_size} px tiles",
            "ms": round(ms, 4), "MPs": round(in_mp / (ms / 1e3), 1),
            "output_MPix_per_frame_ms": round(ms / (d.n_frames * d.out_height * d.out_width / 1e6), 5),
            "kernels_ms": {k: round(v, 4) for k, v in kern.items()},
            "roofline": {"bound": "alu", "kernel": "k_merge", "achieved": round(ach, 3),
                         "peak": round(ALU_PEAK_TOPS, 2), "unit": "Top/s", "frac": round(ach / ALU_PEAK_TOPS, 4),
                         "algorithmic_ops": ops},
            "hbm_frac": round(byts / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}


def bench_stream(burst, out, reps: int = 5) -> dict:
    """The 12 MP x 8 burst merged through the streaming calls: the base frame,
    then one call per aligned frame into a fixed [9][OH][OW] state, then the
    normalisation (each add copies its two frames into the library's
    workspace)."""
    import torch
    from paper_1905_03277_amd import torch_ops

    d = burst.desc
    frames = [burst.frames[k] for k in range(d.n_frames)]
    motion = [burst.motion[k].contiguous() for k in range(d.n_frames)]

    def run():
        sm = torch_ops.StreamingMerge(frames[d.ref_frame], d, burst.tuning)
        for k in range(d.n_frames):
            if k != d.ref_frame:
                sm.add(frames[k], motion[k])
        sm.result(out)

    stream = torch.cuda.current_stream()
    run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        run()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    in_mp = d.n_frames * d.height * d.width / 1e6
    return {"workload": "the 12 MP x 8 burst added frame by frame", "ms": round(ms, 3),
            "MPs": round(in_mp / (ms / 1e3), 1),
            "state_bytes": 9 * 4 * d.out_height * d.out_width}


def align_error_split(burst, motion, frames=(1, 2, 3)) -> dict:
    """Ground-truth error of aligned vectors, split by the base frame's
    structure per tile: the smaller eigenvalue of the Lucas-Kanade normal
    matrix per window pixel, in units of half the noise variance of a
    half-resolution pixel at mid-grey ("flat" < 1, "weak" 1-10, "textured"
    >= 10). Frames 1-3 only (the occluder enters from frame 4)."""
    import numpy as np
    import torch
    d = burst.desc
    f = burst.frames[d.ref_frame].to(torch.float64)
    q = f[0::2, 0::2] + f[0::2, 1::2] + f[1::2, 0::2] + f[1::2, 1::2]
    h, w = q.shape
    xi = torch.arange(w, device=q.device)
    yi = torch.arange(h, device=q.device)
    gx = (q[:, (xi + 1).clamp(max=w - 1)] - q[:, (xi - 1).clamp(min=0)]) / 2.0
    gy = (q[(yi + 1).clamp(max=h - 1), :] - q[(yi - 1).clamp(min=0), :]) / 2.0

    def integral(a):
        z = torch.zeros((h + 1, w + 1), dtype=a.dtype, device=a.device)
        z[1:, 1:] = a.cumsum(0).cumsum(1)
        return z

    B = d.tile_size // 2
    ty = torch.arange(d.tiles_y, device=q.device)
    tx = torch.arange(d.tiles_x, device=q.device)
    y0 = (ty * B - B // 2).clamp(min=0).view(-1, 1)
    y1 = (ty * B + B + B // 2).clamp(max=h).view(-1, 1)
    x0 = (tx * B - B // 2).clamp(min=0).view(1, -1)
    x1 = (tx * B + B + B // 2).clamp(max=w).view(1, -1)

    def box(a):
        z = integral(a)
        return z[y1, x1] - z[y0, x1] - z[y1, x0] + z[y0, x0]

    hxx, hxy, hyy = box(gx * gx), box(gx * gy), box(gy * gy)
    npx = ((y1 - y0) * (x1 - x0)).to(torch.float64)
    lmin = ((hxx + hyy) - torch.sqrt((hxx - hyy) ** 2 + 4 * hxy ** 2)) / 2.0 / npx
    var = 4.0 * (d.noise_a * 0.5 + d.noise_b) * (d.white_level - d.black_level) ** 2
    rel = (lmin / (var / 2.0)).cpu().numpy()
    m = motion.cpu().numpy()
    gt = burst.motion.cpu().numpy()
    res = {}
    for name, lo, hi in (("flat", 0.0, 1.0), ("weak", 1.0, 10.0), ("textured", 10.0, float("inf"))):
        sel = (rel >= lo) & (rel < hi)
        e = np.concatenate([np.hypot(*(m[k] - gt[k])[sel].reshape(-1, 2).T) for k in frames]) if sel.any() else None
        res[name] = {"tiles": round(float(sel.mean()), 3),
                     "median_px": None if e is None else round(float(np.median(e)), 3),
                     "p90_px": None if e is None else round(float(np.percentile(e, 90)), 3)}
    return res


def bench_align(burst, out, reps: int = 10) -> dict:
    """Tile alignment (Sec. 3.2) of the same 12 MP x 8 burst: pyramid, block
    matching on every level, Lucas-Kanade; and raw burst to RGB (alignment then
    merge). Per-stage time from the library's own event timing."""
    import torch
    from paper_1905_03277_amd import binding, torch_ops

    d = burst.desc
    motion = torch.empty_like(burst.motion)

    def al():
        torch_ops.align(burst.frames, d, motion=motion)

    def raw():
        al()
        torch_ops.merge(burst.frames, motion, d, burst.tuning, out=out)

    stream = torch.cuda.current_stream()
    res = {}
    for name, fn in (("align", al), ("raw_to_rgb", raw)):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1) / reps
    binding.hmfsr_profile_begin()
    for _ in range(reps):
        al()
    st = binding.hmfsr_profile_end()
    tot, cnt = st["align"]
    in_mp = d.n_frames * d.height * d.width / 1e6
    tiles = d.tiles_y * d.tiles_x
    alg_bytes = 2 * d.n_frames * d.height * d.width + 8 * d.n_frames * tiles
    al()
    gated = align_error_split(burst, motion)
    ungated = align_error_split(burst, torch_ops.align(burst.frames, d, {"gate": 0.0}))
    return {"workload": "alignment of the 12 MP x 8 burst (4 levels, radii 4/2, 3 Lucas-Kanade "
                        "iterations, noise gate 4, 16 px tiles)",
            "gt_error": {"noise_gate_4": gated, "no_gate": ungated},
            "ms": round(res["align"], 3), "MPs": round(in_mp / (res["align"] / 1e3), 1),
            "stage_ms": round(tot / max(cnt, 1), 3),
            "hbm_algorithmic_bytes": alg_bytes,
            "hbm_frac": round(alg_bytes / (res["align"] / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "raw_to_rgb_ms": round(res["raw_to_rgb"], 3),
            "raw_to_rgb_MPs": round(in_mp / (res["raw_to_rgb"] / 1e3), 1)}


def bench_hf(burst, out, reps: int = 10) -> dict:
    """The same 12 MP x 8 merge with the high-frequency artefact rejection of
    S.3 switched on (hf_ratio 0.02): per-stage times from the library's event
    timing, with the generator's vectors and with the aligner's own."""
    import torch
    from paper_1905_03277_amd import binding, torch_ops

    d = burst.desc
    tun = burst.tuning.replace(hf_ratio=0.02)
    aligned = torch_ops.align(burst.frames, d)
    res = {"workload": "12 MP x 8 merge with S.3 rejection (hf_ratio 0.02)"}
    for name, motion in (("given_vectors", burst.motion), ("aligned_vectors", aligned)):
        torch_ops.merge(burst.frames, motion, d, tun, out=out)
        torch.cuda.synchronize()
        binding.hmfsr_profile_begin()
        for _ in range(reps):
            torch_ops.merge(burst.frames, motion, d, tun, out=out)
        st = binding.hmfsr_profile_end()
        res[name] = {k: round(tot / max(cnt, 1), 4) for k, (tot, cnt) in st.items() if cnt}
    return res


def bench_noise(burst, out, reps: int = 10) -> dict:
    """Noise model: the Monte-Carlo table (64 bins x 4096 patches), the
    12 MP x 8 merge reading it, and the SNR-dependent tuning of the burst."""
    import torch
    from paper_1905_03277_amd import binding, torch_ops

    d = burst.desc
    stream = torch.cuda.current_stream()
    table = torch_ops.noise_table(d, burst.frames.device, bins=64, patches=4096)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        torch_ops.noise_table(d, burst.frames.device, bins=64, patches=4096)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_table = e0.elapsed_time(e1) / reps
    dt = d.replace(noise_table=table)
    torch_ops.merge(burst.frames, burst.motion, dt, burst.tuning, out=out)
    binding.hmfsr_profile_begin()
    for _ in range(reps):
        torch_ops.merge(burst.frames, burst.motion, dt, burst.tuning, out=out)
    st = binding.hmfsr_profile_end()
    t0 = time.perf_counter()
    for _ in range(reps):
        tun, tile, snr = torch_ops.auto_tuning(burst.frames, d)
    ms_tune = (time.perf_counter() - t0) * 1e3 / reps
    return {"table_ms": round(ms_table, 3), "table": "64 bins x 4096 patches x 2 frames x 9 guide px",
            "merge_with_table_kernels_ms": {k: round(tot / max(cnt, 1), 4) for k, (tot, cnt) in st.items() if cnt},
            "auto_tuning_ms_host_clock": round(ms_tune, 3), "snr": round(snr, 2), "suggested_tile": tile,
            "k_detail": round(tun.k_detail, 4)}


def bench_grad(dev, reps: int = 3) -> dict:
    """The differentiation workload: 16 bursts of 8 x 768 x 1024 RGGB at scale 2.
    One pass = for every burst, the forward merge (keeping the normaliser of
    eq. 1), the L2 loss gradient against the synthetic ground-truth scene and
    the adjoint (tuning and motion gradients)."""
    import torch
    from paper_1905_03277_amd import binding, synth, torch_ops

    print("[bench] generating the 16-burst differentiation workload", file=sys.stderr, flush=True)
    bursts = [synth.make_config(5, burst=i, device=dev) for i in range(16)]
    d0 = bursts[0].desc
    outs = [torch.empty((3, b.desc.out_height, b.desc.out_width), dtype=torch.float32, device=dev)
            for b in bursts]
    saveds = [torch_ops.saved_buffer(b.desc, dev)
              for b in bursts]
    grads = []

    def fwd():
        for b, o, sv in zip(bursts, outs, saveds):
            torch_ops.merge(b.frames, b.motion, b.desc, b.tuning, out=o, saved=sv)

    def fwd_bwd():
        grads.clear()
        for b, o, sv in zip(bursts, outs, saveds):
            torch_ops.merge(b.frames, b.motion, b.desc, b.tuning, out=o, saved=sv)
            g = (o - b.gt).mul_(2.0 / o.numel())          # d/dC of mean((C - GT)^2)
            grads.append(torch_ops.merge_backward(b.frames, b.motion, b.desc, b.tuning, g, saved=sv))

    stream = torch.cuda.current_stream()

    def timeit(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    print("[bench] differentiation: forward, forward + adjoint", file=sys.stderr, flush=True)
    ms_f = timeit(fwd)
    ms_fb = timeit(fwd_bwd)
    binding.hmfsr_profile_begin()
    fwd_bwd()
    stages = binding.hmfsr_profile_end()
    loss = float(sum(torch.mean((o - b.gt) ** 2).item() for o, b in zip(outs, bursts)) / len(bursts))
    kern = {k: tot / max(cnt, 1) for k, (tot, cnt) in stages.items()}
    n, hp = d0.n_frames, (d0.height // 2) * (d0.width // 2)
    adj_ops = OPS_ADJ_SAMPLE * n * d0.out_height * d0.out_width + OPS_ADJ_OMEGA * n * hp
    adj_achieved = adj_ops / (kern["k_merge_bwd"] / 1e3) / 1e12
    g_t = torch.stack([g[0] for g in grads]).sum(0).cpu().tolist()
    in_mp = sum(b.desc.n_frames * b.desc.height * b.desc.width for b in bursts) / 1e6
    return {"workload": f"16 bursts, {d0.n_frames} frames {d0.width}x{d0.height} RGGB, scale {d0.scale}, "
                        "L2 loss against the synthetic scene",
            "input_MP": round(in_mp, 1), "ms_fwd": round(ms_f, 3), "ms_fwd_bwd": round(ms_fb, 3),
            "MPs_fwd": round(in_mp / (ms_f / 1e3), 1), "MPs_fwd_bwd": round(in_mp / (ms_fb / 1e3), 1),
            "kernels_ms_per_burst": {k: round(v, 4) for k, v in kern.items()},
            "roofline_adjoint": {"bound": "alu", "kernel": "k_merge_bwd", "achieved": round(adj_achieved, 3),
                                 "peak": round(ALU_PEAK_TOPS, 2), "unit": "Top/s",
                                 "frac": round(adj_achieved / ALU_PEAK_TOPS, 4), "algorithmic_ops": adj_ops},
            "mean_loss": loss,
            "grad_tuning_sum": dict(zip(binding.GRAD_NAMES, [float(f"{v:.6g}") for v in g_t]))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-burst batched leg")
    ap.add_argument("--no-grad", action="store_true", help="skip the forward + adjoint leg")
    ap.add_argument("--no-stream", action="store_true", help="skip the frame-by-frame streaming leg")
    ap.add_argument("--no-align", action="store_true", help="skip the alignment / raw-to-RGB leg")
    ap.add_argument("--no-configs", action="store_true", help="skip the config-3 and config-1 legs")
    ap.add_argument("--only-config", type=int, choices=(1, 3), default=None,
                    help="time only that workload's forward merge (for a profile of it alone) and print its record")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py times the merge on one GPU only (--gpus 1); sharding the merge by "
              "output bands across GPUs is designed but not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1905_03277_amd import synth, torch_ops

    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.only_config is not None:
        print(json.dumps({"only_config": args.only_config, **bench_config(args.only_config, dev, args.steps)}),
              flush=True)
        return
    print("[bench] generating 8x3024x4032 burst", file=sys.stderr, flush=True)
    burst = synth.make_config(2, device=dev)
    d = burst.desc
    out = torch.empty((3, d.out_height, d.out_width), dtype=torch.float32, device=dev)

    def step():
        torch_ops.merge(burst.frames, burst.motion, d, burst.tuning, out=out)

    calibration_copy(dev)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("[bench] timing", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / args.steps

    # per-kernel durations: a second pass with the library's event timing on
    from paper_1905_03277_amd import binding
    binding.hmfsr_profile_begin()
    for _ in range(args.steps):
        step()
    stages = binding.hmfsr_profile_end()
    kern_ms = {k: tot / max(cnt, 1) for k, (tot, cnt) in stages.items()}

    in_mp = d.n_frames * d.height * d.width / 1e6
    value = in_mp / (ms / 1e3)
    ops = algorithmic_ops(d)
    byts = algorithmic_bytes(d)
    dom = "k_merge"
    achieved = ops[dom] / (kern_ms[dom] / 1e3) / 1e12
    line = {
        "metric": "merge input-Bayer MP/s at 12MP x 8 fwd",
        "value": round(value, 1),
        "unit": "MP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": "forward merge, 8 frames 4032x3024 RGGB uint16 12-bit, occluder, "
                               "scale 1, 16 px tiles", "frames": d.n_frames, "height": d.height,
                   "width": d.width, "scale": d.scale},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(ALU_PEAK_TOPS, 2),
                     "unit": "Top/s", "frac": round(achieved / ALU_PEAK_TOPS, 4), "traffic": measured_traffic(),
                     "kernel": dom, "kernel_ms": round(kern_ms[dom], 4),
                     "algorithmic_ops": ops[dom]},
        "kernels_ms": {k: round(v, 4) for k, v in kern_ms.items()},
        "hbm": {"algorithmic_bytes": byts["total"],
                "achieved_GBs": round(byts["total"] / (ms / 1e3) / 1e9, 1),
                "peak_GBs": HBM_PEAK_GBS,
                "frac": round(byts["total"] / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
        "wall_s_timed": round(wall, 3),
    }
    if not args.no_configs:
        line["config3_low_light"] = bench_config(3, dev)
        line["config1_small"] = bench_config(1, dev)
    if not args.no_stream:
        line["streaming"] = bench_stream(burst, out)
    if not args.no_align:
        line["alignment"] = bench_align(burst, out)
        line["hf_rejection"] = bench_hf(burst, out)
        line["noise_model"] = bench_noise(burst, out)
    if not args.no_batch:
        line["batched"] = bench_batch(dev)
    if not args.no_grad:
        line["fwd_bwd"] = bench_grad(dev)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(burst.to("cpu"))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
