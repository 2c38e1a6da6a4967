"""Benchmark of the inpainting hot path on one MI355X.

A step is one complete inpainting of one clip: context creation (pyramids,
texture features, sets), onion-peel initialisation, the EM loop of every
level (ANN search + weighted reconstruction, 20 iterations per level),
level transitions and the final best-patch reconstruction, from the input
video resident in HBM to the output video in HBM.  The headline workload is
the HD clip (1920x1080 px x 60 frames, 5-level pyramid, the largest
single-GPU configuration); the SD clip (854x480 px x 100 frames, 4 levels)
is measured in the same run and reported under "sd".

Prints one JSON line.  `value` is nominal NNF patch-distance evaluations per
second over the timed steps (the nominal count of a search is |H~| x (1 + sum
over iterations of 6 n_jf + [radius >= 1]) and does not depend on how many
candidates an implementation skips).  The roofline object covers the
propagation-pass kernel, timed with HIP events on the context's stream over
the timed steps (one event pair around the back-to-back passes of each
search; the average launch duration is their time over their count); its
binding roof is the one the hardware counters of the same kernel show
nearer to saturation (HBM traffic against the device's measured copy rate, or VALU
issue).  The CPU baseline is the oracle's search over a sample of the
finest level's targets of the same clip, on all host cores and on one.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: int32 VALU lane operations per second
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
BYTES_PER_EVAL = 625  # 125 voxels x 5 uint8 channels of the candidate patch
# per target and pass: its own patch through the workgroup's tile (5 B) and
# the shift-map state (six 4-byte neighbour reads, one 8-byte write)
BYTES_PER_TARGET_PASS = 37
OPS_PER_EVAL = 1250  # 625 subtractions + 625 multiply-adds (5 channels x 125 voxels)
MFMA_INT8_PEAK_TOPS = 5000.0  # dense 8-bit matrix-core peak, TOP/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="hd", choices=["sd", "hd", "tiny"])
    ap.add_argument("--no-realign", action="store_true",
                    help="skip the realignment measurement (Sec. 3.4)")
    ap.add_argument("--reduce-dims", type=int, default=0,
                    help="run the main workload in the PCA-reduced patch space (profiling; "
                         "the headline is the exact method)")
    ap.add_argument("--appb-only", action="store_true",
                    help="only the textured-patch experiment (App. B), then exit")
    ap.add_argument("--no-reduced", action="store_true",
                    help="skip the PCA-reduced patch space measurement (Sec. 5)")
    ap.add_argument("--no-image", action="store_true",
                    help="skip the 2-D image inpainting measurement")
    ap.add_argument("--no-appb", action="store_true",
                    help="skip the textured-patch experiment (App. B)")
    ap.add_argument("--no-sd", action="store_true",
                    help="skip the SD clip measured beside the headline workload")
    ap.add_argument("--sd-steps", type=int, default=3)
    ap.add_argument("--em-iters", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-frames", type=int, default=60,
                    help="frames of the crop whose finest level the all-core oracle sample "
                         "searches")
    ap.add_argument("--cpu-frames-1core", type=int, default=10,
                    help="frames of the crop the one-core oracle sample searches")
    ap.add_argument("--cpu-sample-run", nargs=2, metavar=("CONFIG", "FRAMES"),
                    help=argparse.SUPPRESS)
    ap.add_argument("--oracle-timing", action="store_true",
                    help="time the oracle on one host core and on all of them and exit")
    ap.add_argument("--oracle-timing-run", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--batch-clips", type=int, default=64)
    ap.add_argument("--served-seconds", type=float, default=30.0)
    ap.add_argument("--served-rate", type=float, default=4.0)
    ap.add_argument("--served-sweep", metavar="RATES",
                    help="comma-separated arrival rates (jobs/s; 0 = all jobs at once): served "
                         "against serial FIFO on Poisson traces of --served-jobs jobs, then exit")
    ap.add_argument("--served-jobs", type=int, default=240)
    ap.add_argument("--summarize-counters", metavar="DIR",
                    help="summarise a rocprofv3 --output-format csv directory and exit")
    ap.add_argument("--assemble-counters", nargs=5,
                    metavar=("PASS_FETCH", "PASS_WRITE", "PASS_SQ", "COPY_FETCH", "COPY_WRITE"),
                    help="write the search kernel's HBM traffic record from four "
                         "--summarize-counters outputs (JSON files) and exit")
    return ap.parse_args()


KERNEL_SRC = os.path.join(ROOT, "paper_1503_05528_amd", "csrc", "vi_kernels.hip")


def counters_json(workload):
    return os.path.join(ROOT, "profiles", f"k_pass_{workload}_counters.json")


def log(msg):
    """Progress line on stderr (the JSON result line goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    import hashlib
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()


def summarize_counters(d):
    """Per kernel and grid size: dispatches, mean duration and mean value of
    every counter of a rocprofv3 CSV output directory."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        rows += list(csv.DictReader(open(f)))
    agg = {}
    for r in rows:
        k = (r["Kernel_Name"].split("(")[0].replace("void ", ""), int(r["Grid_Size"]))
        a = agg.setdefault(k, {"dispatch": {}, "counters": {}})
        a["dispatch"][r["Dispatch_Id"]] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        a["counters"].setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    out = []
    for (name, grid), a in sorted(agg.items()):
        ds = list(a["dispatch"].values())
        out.append({"kernel": name, "grid": grid, "dispatches": len(ds),
                    "mean_us": sum(ds) / len(ds) / 1000.0,
                    "counters": {c: sum(v) / len(v) for c, v in sorted(a["counters"].items())}})
    return out


# the exact-distance search pass: one template, instantiated for the passes
# with the random search fused (every third pass) and for the others
PASS_KERNELS = ("vi::k_pass<false, false, false>", "vi::k_pass<false, false, true>")
COPY_KERNEL = "__amd_rocclr_copyBuffer"
COPY_BYTES = 1 << 30
SQ_COUNTERS = "SQ_WAVES SQ_INSTS_VALU SQ_INSTS_VMEM_RD SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT GRBM_GUI_ACTIVE"


def assemble_counters(pass_fetch, pass_write, pass_sq, copy_fetch, copy_write, workload):
    """The search kernel's counter record: HBM bytes per launch from
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch, averaged over every
    dispatch of the kernel at every grid size) scaled by what the same
    counters read for a plain 1 GiB device copy, which reads and writes
    exactly COPY_BYTES; VALU issue from SQ_INSTS_VALU (wave instructions; a
    CU issues at most one per cycle across its four SIMDs) over the
    dispatch's cycles at 2.4 GHz on 256 CUs."""
    def load(path, kernels):
        rows = [r for r in json.load(open(path)) if r["kernel"] in kernels]
        n = sum(r["dispatches"] for r in rows)
        if n == 0:
            raise SystemExit(f"{path}: no dispatch of {kernels}")
        return rows, n

    def mean(rows, n, counter):
        return sum(r["counters"][counter] * r["dispatches"] for r in rows) / n

    def mean_us(rows, n):
        return sum(r["mean_us"] * r["dispatches"] for r in rows) / n
    rf, nf = load(pass_fetch, PASS_KERNELS)
    rw, nw = load(pass_write, PASS_KERNELS)
    rs, ns = load(pass_sq, PASS_KERNELS)
    cf_rows, cfn = load(copy_fetch, (COPY_KERNEL,))
    cw_rows, cwn = load(copy_write, (COPY_KERNEL,))
    fk, wk = mean(rf, nf, "FETCH_SIZE"), mean(rw, nw, "WRITE_SIZE")
    cf, cw = mean(cf_rows, cfn, "FETCH_SIZE"), mean(cw_rows, cwn, "WRITE_SIZE")
    fscale = COPY_BYTES / 1024.0 / cf
    wscale = COPY_BYTES / 1024.0 / cw
    us = mean_us(rf, nf)
    sq = {c: mean(rs, ns, c) for c in SQ_COUNTERS.split()}
    sq_us = mean_us(rs, ns)
    per_level = []
    for r in sorted(rf, key=lambda r: (-r["grid"], r["kernel"])):
        key = (r["kernel"], r["grid"])
        w = next((x for x in rw if (x["kernel"], x["grid"]) == key), None)
        q = next((x for x in rs if (x["kernel"], x["grid"]) == key), None)
        hb = 1024.0 * (r["counters"]["FETCH_SIZE"] * fscale
                       + (w["counters"]["WRITE_SIZE"] * wscale if w else 0.0))
        per_level.append({
            "kernel": r["kernel"], "grid": r["grid"], "dispatches": r["dispatches"],
            "mean_us": r["mean_us"],
            "hbm_bytes_per_launch": hb, "hbm_gbs": hb / (r["mean_us"] * 1e-6) / 1e9,
            "valu_busy": (q["counters"]["SQ_INSTS_VALU"] / (256 * q["mean_us"] * 2400.0)
                          if q else None)})
    rec = {
        "kernel": list(PASS_KERNELS), "workload": workload,
        "source_sha256": kernel_source_hash(),
        "fetch_kib_per_launch": fk, "write_kib_per_launch": wk,
        "fetch_scale": fscale, "write_scale": wscale,
        "hbm_bytes_per_launch": 1024.0 * (fk * fscale + wk * wscale),
        "mean_launch_us": us, "dispatches": nf,
        "sq_per_launch": sq, "sq_mean_launch_us": sq_us,
        "valu_busy": sq["SQ_INSTS_VALU"] / (256 * sq_us * 2400.0),
        "per_grid": per_level,
        "copy_calibration": {"bytes": COPY_BYTES, "FETCH_SIZE_kib": cf, "WRITE_SIZE_kib": cw,
                             "mean_us": mean_us(cf_rows, cfn)},
        "commands": [
            f"cd /tmp && TMPDIR=/tmp rocprofv3 --pmc FETCH_SIZE --kernel-include-regex k_pass "
            f"--output-format csv -d /tmp/p_FETCH_SIZE -o run -- python $REPO/bench.py "
            f"--config {workload} --no-sd --no-cpu-baseline --no-batched --no-served "
            f"--no-realign --no-appb --no-image --no-reduced --steps 1 --warmup 0",
            "(the same with --pmc WRITE_SIZE, and with --pmc " + SQ_COUNTERS + ")",
            "cd /tmp && TMPDIR=/tmp rocprofv3 --pmc FETCH_SIZE --output-format csv "
            "-d /tmp/c_FETCH_SIZE -o run -- python $REPO/bench.py --copy-calibration "
            "(and the same with WRITE_SIZE)",
            "python $REPO/bench.py --summarize-counters <dir> > <json>   (each of the five)",
            "python $REPO/bench.py --config " + workload + " --assemble-counters <pass FETCH> "
            "<pass WRITE> <pass SQ> <copy FETCH> <copy WRITE>",
        ],
    }
    with open(counters_json(workload), "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    return rec


def _gen_batch_clip(seed):
    from paper_1503_05528_amd import synth
    c = synth.batch_clip(seed)
    return c.occluded_input(), c.mask, c.levels


def gen_batch_clips(n, base_seed=1000):
    """The mixed-size batch workload, generated in worker processes."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    with ctx.Pool(min(8, max(1, os.cpu_count() or 1))) as pool:
        return pool.map(_gen_batch_clip, [base_seed + i for i in range(n)])


def batched_vs_serial(clips, em_iters):
    """One clip at a time (vi_inpaint) versus all clips in one batch (one
    graph launch per EM iteration), from inputs resident in HBM to outputs
    in HBM; outputs must be identical."""
    import torch
    from paper_1503_05528_amd import vi
    dev = [(torch.from_numpy(v).cuda(), torch.from_numpy(m).cuda(), L) for v, m, L in clips]
    mk = lambda i: vi.default_params(levels=dev[i][2], em_tol=-1.0, em_max_iters=em_iters,
                                     seed=1000 + i)
    # warm-up (kernels, allocator)
    g = vi.Clip(dev[0][0], dev[0][1], params=mk(0))
    g.inpaint()
    g.close()
    torch.cuda.synchronize()
    serial_out, service = [], []
    nominal = 0
    log(f"batched: {len(dev)} clips one at a time")
    t0 = time.perf_counter()
    for i, (v, m, L) in enumerate(dev):
        s0 = time.perf_counter()
        g = vi.Clip(v, m, params=mk(i))
        serial_out.append(g.inpaint())
        nominal += g.counters()["nominal_evals"]
        g.close()
        service.append(time.perf_counter() - s0)
    torch.cuda.synchronize()
    t_serial = time.perf_counter() - t0
    log("batched: tuning on a throw-away batch")
    b = vi.Batch()
    # tune once on a throw-away batch of the same clips so the timed run
    # measures steady-state steps
    tb = [vi.Clip(v, m, params=mk(i)) for i, (v, m, L) in enumerate(dev)]
    for g in tb:
        b.add(g)
    b.step()
    tune = b.tune()
    for g in tb:
        g.close()
    b.close()
    torch.cuda.synchronize()
    log(f"batched: all clips in one batch, tune {tune}")
    t0 = time.perf_counter()
    b = vi.Batch(tune=tune)
    members = [vi.Clip(v, m, params=mk(i)) for i, (v, m, L) in enumerate(dev)]
    for g in members:
        b.add(g)
    steps = b.run()
    outs = [g.output() for g in members]
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    same = all(torch.equal(a, c) for a, c in zip(outs, serial_out))
    for g in members:
        g.close()
    b.close()
    n = len(dev)
    return {"clips": n, "serial_clips_per_s": n / t_serial, "batched_clips_per_s": n / t_batch,
            "speedup": t_serial / t_batch, "serial_s": t_serial, "batched_s": t_batch,
            "batched_steps": steps, "tune": list(tune) if tune else None,
            "outputs_identical": bool(same), "nominal_evals": nominal,
            "batched_evals_per_s": nominal / t_batch}, service


def host_service_times(clips, sd_clip, idxs, em_iters):
    """Serial service time of each clip as a request sees it: input from host
    memory to the device, context, inpainting, output back to host memory
    (index -1: the SD clip)."""
    import torch
    from paper_1503_05528_amd import vi
    out = {}
    for idx in [idxs[0]] + list(idxs):  # the first run also warms up
        v, m, L = sd_clip if idx < 0 else clips[idx]
        torch.cuda.synchronize()
        s = time.perf_counter()
        g = vi.Clip(torch.from_numpy(v).cuda(), torch.from_numpy(m).cuda(), levels=L,
                    em_tol=-1.0, em_max_iters=em_iters, seed=1)
        g.inpaint().cpu()
        g.close()
        out[idx] = time.perf_counter() - s
    return out


def served(clips, sd_clip, seconds, rate, em_iters, service_alone):
    """Poisson arrivals served by the continuous-batching server, against
    serial FIFO execution of the same trace: with each clip's serial service
    time through host memory, as the server's requests arrive and leave, and
    (for reference) with the device-resident service times service_alone."""
    import threading
    import torch
    from paper_1503_05528_amd import synth
    from paper_1503_05528_amd.serve import GpuEngine, Request, Server, fifo_latencies, percentile
    trace = synth.served_trace(seconds, rate, seed=2000)
    rng = __import__("numpy").random.default_rng(7)
    jobs = []
    for (t, kind, seed) in trace:
        if kind == "sd":
            jobs.append((t, -1))
        else:
            jobs.append((t, int(rng.integers(0, len(clips)))))
    log("served: serial service times through host memory")
    host_svc = host_service_times(clips, sd_clip, sorted({i for _, i in jobs}), em_iters)
    free = torch.cuda.mem_get_info()[0]
    # two lanes: clips of up to 20 M voxels, and larger ones, overlap on the GPU
    lanes = [GpuEngine(), GpuEngine()]
    big = lambda r: 1 if r.mask.size > 20_000_000 else 0
    srv = Server(lanes, hbm_budget=int(0.8 * free), max_slots=256, route=big)

    def req(idx):
        if idx < 0:
            v, m, L = sd_clip
        else:
            v, m, L = clips[idx]
        return Request(v, m, dict(levels=L, em_tol=-1.0, em_max_iters=em_iters, seed=1),
                       hole_fraction=float(m.mean()))
    srv.start()
    t0 = time.perf_counter()
    futs = []

    def feeder():
        for (t, idx) in jobs:
            d = t0 + t - time.perf_counter()
            if d > 0:
                time.sleep(d)
            r = req(idx)
            r.arrival = t0 + t
            futs.append(srv.submit(r))
    th = threading.Thread(target=feeder)
    th.start()
    th.join()
    for f in futs:
        f.result()
    t_end = time.perf_counter()
    srv.stop()
    for e in lanes:
        e.close()
    st = srv.latency_stats()
    serial = fifo_latencies([t for t, _ in jobs], [host_svc[idx] for _, idx in jobs])
    serial_dev = fifo_latencies([t for t, _ in jobs], [service_alone[idx] for _, idx in jobs])
    return {"rate_per_s": rate, "duration_s": seconds, "jobs": len(jobs),
            "sd_jobs": sum(1 for _, i in jobs if i < 0),
            "clips_per_s": len(jobs) / (t_end - t0),
            "p50_s": st.get("p50_s"), "p99_s": st.get("p99_s"),
            "serial_fifo_p50_s": percentile(serial, 0.5),
            "serial_fifo_p99_s": percentile(serial, 0.99),
            "serial_fifo_device_resident_p50_s": percentile(serial_dev, 0.5),
            "serial_fifo_device_resident_p99_s": percentile(serial_dev, 0.99),
            "max_running": srv.max_running, "steps": srv.steps,
            "max_admitted_gb": srv.max_admitted_bytes / 2 ** 30}


def served_sweep(rates, n_jobs, em_iters):
    """Served capacity: for each arrival rate, a Poisson trace of n_jobs jobs
    (90 % batch-mix clips, 10 % SD) through the continuous-batching server,
    against serial FIFO execution of the same trace with each clip's serial
    service time through host memory.  Rate 0: every job arrives at once
    (the server's and the serial path's throughput at saturation)."""
    import threading
    import numpy as np
    import torch
    from paper_1503_05528_amd.serve import GpuEngine, Request, Server, fifo_latencies
    bclips = gen_batch_clips(64)
    sd, L = make_clip("sd")
    sd_clip = (sd.occluded_input(), sd.mask, L)
    log("served sweep: serial service times through host memory")
    svc = host_service_times(bclips, sd_clip, [-1] + list(range(len(bclips))), em_iters)
    rows = []
    for rate in rates:
        rng = np.random.default_rng(2000 + int(rate * 10))
        t, jobs = 0.0, []
        for _ in range(n_jobs):
            if rate > 0:
                t += rng.exponential(1.0 / rate)
            jobs.append((t, -1 if rng.uniform() < 0.10 else int(rng.integers(0, len(bclips)))))
        free = torch.cuda.mem_get_info()[0]
        lanes = [GpuEngine(), GpuEngine()]
        srv = Server(lanes, hbm_budget=int(0.8 * free), max_slots=256,
                     route=lambda r: 1 if r.mask.size > 20_000_000 else 0)

        def req(idx):
            v, m, Lv = sd_clip if idx < 0 else bclips[idx]
            return Request(v, m, dict(levels=Lv, em_tol=-1.0, em_max_iters=em_iters, seed=1),
                           hole_fraction=float(m.mean()))
        log(f"served sweep: {n_jobs} jobs at {rate} jobs/s")
        srv.start()
        t0 = time.perf_counter()
        futs = []

        def feeder():
            for (ta, idx) in jobs:
                d = t0 + ta - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                r = req(idx)
                r.arrival = t0 + ta
                futs.append(srv.submit(r))
        th = threading.Thread(target=feeder)
        th.start()
        th.join()
        for f in futs:
            f.result()
        t_end = time.perf_counter()
        srv.stop()
        for e in lanes:
            e.close()
        lat = sorted(r.latency for r in srv.records if r.ok)
        arrivals = [ta for ta, _ in jobs]
        serial = fifo_latencies(arrivals, [svc[idx] for _, idx in jobs])
        serial_end = max(a + l for a, l in zip(arrivals, serial))
        rows.append({
            "rate_per_s": rate, "jobs": n_jobs, "sd_jobs": sum(1 for _, i in jobs if i < 0),
            "served_clips_per_s": n_jobs / (t_end - t0),
            "served_p50_s": percentile(lat, 0.5), "served_p99_s": percentile(lat, 0.99),
            "serial_clips_per_s": n_jobs / serial_end,
            "serial_p50_s": percentile(serial, 0.5), "serial_p99_s": percentile(serial, 0.99),
            "max_running": srv.max_running, "steps": srv.steps})
        log(json.dumps(rows[-1]))
    mean_svc = sum(svc[i] for i in range(len(bclips))) * 0.9 / len(bclips) + 0.1 * svc[-1]
    return {"served_sweep": rows, "serial_capacity_clips_per_s": 1.0 / mean_svc,
            "mean_serial_service_s": mean_svc}


def measure_realign(steps=3):
    """Realignment of a shaking-camera clip (854x480 px x 50 frames):
    estimation of every frame pair's motion, composition, warp of video and
    occlusion, unwarp into the occlusion; GPU times (inputs resident in
    HBM)."""
    import numpy as np
    import torch
    from paper_1503_05528_amd import synth, vi
    clip, cams = synth.jittered(seed=11, W=854, H=480, T=50)
    T, H, W, _ = clip.video.shape
    v = torch.from_numpy(clip.occluded_input()).cuda()
    m = torch.from_numpy(clip.mask).cuda()
    aligned = torch.from_numpy(clip.video).cuda()
    theta = vi.align_estimate(v, m)  # warm-up
    M = vi.align_compose(theta, T)
    vi.align_warp(v, m, M)
    torch.cuda.synchronize()
    t_est, t_warp, t_unwarp = [], [], []
    for _ in range(steps):
        s0 = time.perf_counter()
        theta = vi.align_estimate(v, m)
        M = vi.align_compose(theta, T)
        s1 = time.perf_counter()
        av, am = vi.align_warp(v, m, M)
        torch.cuda.synchronize()
        s2 = time.perf_counter()
        out = vi.align_unwarp(aligned, v, m, M)
        torch.cuda.synchronize()
        s3 = time.perf_counter()
        t_est.append(s1 - s0)
        t_warp.append(s2 - s1)
        t_unwarp.append(s3 - s2)
    est, warp, unwarp = (statistics.median(x) for x in (t_est, t_warp, t_unwarp))
    # truth: the cameras' exact inter-frame motion, corner error in px
    def h3(q):
        return np.array([[q[0], q[1], q[2]], [q[3], q[4], q[5]], [0, 0, 1.0]])
    cn = np.array([[0, 0, 1], [W - 1, 0, 1], [0, H - 1, 1], [W - 1, H - 1, 1.0]]).T
    err = max(np.abs(((np.linalg.inv(h3(cams[n + 1])) @ h3(cams[n])) @ cn - h3(theta[n]) @ cn)[:2]).max()
              for n in range(T - 1))
    px = W * H * T
    # warp: per output pixel the source frame's 3 colour bytes and mask byte
    # (the 2x2 stencil overlaps its neighbours') and 4 bytes written
    warp_bytes = 8 * px
    return {"workload": f"shaking-camera clip {W}x{H}x{T}, 3 estimation levels x 8 robust "
                        "Gauss-Newton steps per frame pair",
            "estimate_ms": 1000 * est, "warp_ms": 1000 * warp, "unwarp_ms": 1000 * unwarp,
            "frames_per_s": T / (est + warp + unwarp),
            "max_corner_error_px": float(err),
            "warp_call_gbs": warp_bytes / warp / 1e9,
            "warp_call_frac_of_hbm_peak": warp_bytes / warp / 1e9 / HBM_PEAK_GBS}


def measure_image(steps=3, em_iters=20):
    """2-D image inpainting with 5x5x1 patches (T = 1) on the same kernels:
    whole inpaintings of a 1920x1080 and a 3840x2160 still image from
    inputs resident in HBM (the hole about 5 % of the pixels)."""
    import torch
    from paper_1503_05528_amd import synth, vi
    res = []
    for W, H, levels in ((1920, 1080, 5), (3840, 2160, 6)):
        img = synth.image(31, W, H, frac=0.05, levels=levels)
        video = torch.from_numpy(img.occluded_input()).cuda()
        mask = torch.from_numpy(img.mask).cuda()
        params = vi.default_params(levels=levels, em_tol=-1.0, em_max_iters=em_iters, seed=1,
                                   patch=(5, 5, 1))

        def one():
            g = vi.Clip(video, mask, params=params)
            g.inpaint()
            c = g.counters()
            g.close()
            return c
        one()
        torch.cuda.synchronize()
        lat, nominal = [], 0
        for _ in range(steps):
            s0 = time.perf_counter()
            nominal += one()["nominal_evals"]
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - s0)
        res.append({"image": f"{W}x{H}", "levels": levels,
                    "hole_fraction": float(img.mask.mean()),
                    "ms_per_image": 1000 * statistics.median(lat),
                    "nominal_evals_per_s": nominal / sum(lat)})
    return {"workload": "still images, 5x5x1 patches, 20 EM iterations per level", "rows": res}


def image_cpu_baseline():
    """CPU baseline leg of the image workload: the oracle's search of the
    1920x1080 image's finest level (every target, matches drawn at random
    first), on all host cores."""
    from oracle import vio
    from paper_1503_05528_amd import synth
    img = synth.image(31, 1920, 1080, frac=0.05, levels=5)
    o = vio.Oracle(img.occluded_input(), img.mask, levels=5, patch=(5, 5, 1), seed=1)
    (_, _, _), (_, nS, _) = o.info(0)
    c0 = time.perf_counter()
    o.nnf_search(0, 0)
    dt = time.perf_counter() - c0
    # nominal evaluations of one search: |H~| (1 + sum_k (6 n_jf + [radius >= 1]))
    r_max = 1920
    per = 1 + sum(6 * 3 + (1 if int(r_max * 0.5 ** k) >= 1 else 0) for k in range(1, 11))
    return {"value": nS * per / dt, "unit": "evals/s", "cores": vio.num_threads(),
            "kind": "oracle",
            "sample": f"vio_nnf_search of the 1920x1080 image's finest level ({nS} targets)"}


def realign_cpu_baseline():
    """CPU baseline leg of the realignment: the oracle's estimation and warp
    of the same clip on all host cores."""
    from oracle import vio
    from paper_1503_05528_amd import synth
    clip, _ = synth.jittered(seed=11, W=854, H=480, T=50)
    T = clip.video.shape[0]
    vn, mn = clip.occluded_input(), clip.mask
    c0 = time.perf_counter()
    oth = vio.align_estimate(vn, mn)
    c1 = time.perf_counter()
    vio.align_warp(vn, mn, vio.align_compose(oth, T))
    c2 = time.perf_counter()
    return {"kind": "oracle", "estimate_s": c1 - c0, "warp_s": c2 - c1,
            "cores": vio.num_threads(), "sample": "the whole clip"}


# App. B table: probability that a random patch beats the constant patch
# (white noise of grey-level variance 25), as printed
APPB_PRINTED = [((3, 3, 1), 8e-2), ((5, 5, 1), 1e-2), ((3, 3, 3), 6e-3), ((7, 7, 1), 4.1e-4),
              ((9, 9, 1), 5.5e-6), ((11, 11, 1), 3e-7), ((5, 5, 5), 2e-7)]
APPB_SIDE = 256
APPB_REFS = 4096


def measure_appb(steps=3):
    """The textured-patch experiment of App. B: for each of the table's seven
    patch sizes, 4096 white-noise reference patches against every patch of
    a 256^3 white-noise volume (2-D sizes: every patch of each of its 256
    frames), counting the patches closer to the reference than the
    constant patch; GPU time of the call (HIP events on the stream it is
    enqueued on, inputs resident in HBM)."""
    import math
    import numpy as np
    import torch
    from paper_1503_05528_amd import synth, vi
    n = APPB_SIDE
    vol = torch.from_numpy(synth.noise(170, (n, n, n))).cuda()
    rows = []
    total_pairs, total_s = 0, 0.0
    for patch, printed in APPB_PRINTED:
        pw, ph, pt = patch
        N = pw * ph * pt
        n_cand = (n - pw + 1) * (n - ph + 1) * (n - pt + 1)
        ref = torch.from_numpy(synth.noise(1000 + N, (APPB_REFS, pt, ph, pw))).cuda()
        out = vi.closer_than_constant(ref, vol, patch)  # warm-up
        torch.cuda.synchronize()
        ms = []
        for _ in range(steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            vi.closer_than_constant(ref, vol, patch, out=out)
            e1.record()
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        t = statistics.median(ms) / 1000.0
        c = out.cpu().numpy().astype(np.float64)
        rate = c / n_cand
        pairs = APPB_REFS * n_cand
        total_pairs += pairs
        total_s += t
        # per pair: 2 x 64 x ceil(N / 64) 8-bit matrix-core operations (the
        # inner product over the zero-padded 64-byte blocks), and 4 VALU lane
        # operations for the comparison (shift, subtract, compare, add)
        mfma_ops = 128 * ((N + 63) // 64)
        ops = 4
        rows.append({"patch": "x".join(map(str, patch)), "voxels": N, "references": APPB_REFS,
                     "candidates": n_cand, "hits": int(c.sum()), "probability": rate.mean(),
                     "std_error": rate.std(ddof=1) / math.sqrt(APPB_REFS),
                     "paper": printed, "ms": 1000 * t, "pairs_per_s": pairs / t,
                     "valu_frac": pairs / t * ops / (VALU_PEAK_TOPS * 1e12),
                     "mfma_int8_frac": pairs / t * mfma_ops / (MFMA_INT8_PEAK_TOPS * 1e12)})
    return {"workload": f"{n}x{n}x{n} grey white noise (variance 25), {APPB_REFS} reference "
                        "patches per patch size, the seven sizes of the App. B table",
            "pairs_per_s": total_pairs / total_s, "ms_total": 1000 * total_s, "rows": rows,
            "roofline": {"bound": "alu", "unit": "TOP/s", "peak": VALU_PEAK_TOPS,
                         "note": "the comparison's 4 VALU lane operations per pair bind "
                                 "before the 8-bit matrix cores (valu_frac against "
                                 "mfma_int8_frac per row)"}}


def appb_cpu_baseline():
    """CPU baseline leg of App. B: the oracle's brute-force count for one
    5x5x5 reference patch over the whole 256^3 volume."""
    from oracle import vio
    from paper_1503_05528_amd import synth
    n = APPB_SIDE
    vol = synth.noise(170, (n, n, n))
    ref = synth.noise(1000 + 125, (1, 5, 5, 5))
    c0 = time.perf_counter()
    vio.closer_than_constant(ref, vol, (5, 5, 5))
    dt = time.perf_counter() - c0
    return {"value": (n - 4) ** 3 / dt, "unit": "pairs/s", "cores": vio.num_threads(),
            "kind": "oracle", "sample": "one 5x5x5 reference against every patch of the volume"}


def make_clip(name):
    from paper_1503_05528_amd import synth
    if name == "sd":
        return synth.sd(), 4
    if name == "hd":
        return synth.hd(), 5
    return synth.tiny(), 1


# crops (x0, x1, y0, y1) around an occlusion of each clip, for the oracle's
# timing samples
CPU_CROPS = {"hd": (240, 600, 160, 340), "sd": (220, 640, 170, 310), "tiny": (0, 32, 0, 32)}


def cpu_sample_run(config, frames):
    """One process's oracle timing (its OpenMP thread count comes from the
    environment): a complete ANN search of the finest level of a crop of the
    clip (its frames [0, frames) and the CPU_CROPS window, same pyramid
    depth), from the unset shift map (random initialisation, then every
    iteration; the oracle evaluates every candidate in full, so its cost
    does not depend on the state)."""
    import numpy as np
    from oracle import vio
    clip, levels = make_clip(config)
    x0, x1, y0, y1 = CPU_CROPS[config]
    video = np.ascontiguousarray(clip.occluded_input()[:frames, y0:y1, x0:x1])
    mask = np.ascontiguousarray(clip.mask[:frames, y0:y1, x0:x1])
    o = vio.Oracle(video, mask, levels=levels, em_tol=-1.0, seed=1)
    (W, H, T), (_, nS, _) = o.info(0)
    p = o.params
    per = 1
    rmax = max(W, H, T)
    for k in range(1, p.pm_iters + 1):
        r = float(rmax)
        for _ in range(k):
            r *= p.rho
        per += 6 * p.n_jf + (1 if int(r // 1) >= 1 else 0)
    t0 = time.perf_counter()
    o.nnf_search(0, 0)
    dt = time.perf_counter() - t0
    print(json.dumps({"threads": vio.num_threads(), "targets": nS, "evals": per * nS,
                      "seconds": dt, "dims": [W, H, T], "crop": [x0, x1, y0, y1]}), flush=True)


def cpu_baseline(config, frames_all, frames_one):
    """The oracle, as it stands, on a bounded sample of the workload: the
    complete finest-level search of a crop of the clip around an occlusion,
    on all host threads, and of a shorter crop on one thread."""
    import subprocess
    out = {}
    for key, n, fr in (("all", os.cpu_count() or 1, frames_all), ("one", 1, frames_one)):
        env = dict(os.environ, OMP_NUM_THREADS=str(n))
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-sample-run",
                            config, str(fr)], env=env, capture_output=True, text=True,
                           check=True)
        out[key] = json.loads(r.stdout.strip().splitlines()[-1])
    a, b = out["all"], out["one"]
    x0, x1, y0, y1 = a["crop"]

    def desc(r):
        W, H, T = r["dims"]
        return (f"vio_nnf_search of the finest level of the {config} clip cropped to "
                f"x {x0}-{x1 - 1}, y {y0}-{y1 - 1}, frames 0-{T - 1} ({W}x{H}x{T}, "
                f"{r['targets']} targets): {r['evals']} nominal evals in {r['seconds']:.1f} s")
    return {"value": a["evals"] / a["seconds"], "unit": "evals/s", "cores": a["threads"],
            "kind": "oracle", "sample": desc(a),
            "one_core": {"value": b["evals"] / b["seconds"], "unit": "evals/s", "cores": 1,
                         "sample": desc(b)}}


def oracle_timing_run():
    """One process's oracle timings (its OpenMP thread count comes from the
    environment): an ANN search at SD level 1, a weighted reconstruction of
    every SD level-0 hole pixel from a fixed valid shift map, a complete
    inpainting of the tiny clip."""
    import numpy as np
    from oracle import vio
    from paper_1503_05528_amd import synth
    out = {"threads": vio.num_threads()}
    sd = synth.sd()
    o = vio.Oracle(sd.occluded_input(), sd.mask, levels=4, em_tol=-1.0, em_max_iters=20, seed=1)
    (_, _, _), (_, nS1, _) = o.info(1)
    t0 = time.perf_counter()
    o.nnf_search(1, 0)
    out["sd_l1_search_s"] = time.perf_counter() - t0
    out["sd_l1_targets"] = nS1
    hole, dsrc, htil = o.sets(0)
    rgbt, cand, dist, nvox = o.get_state(0)
    rng = np.random.default_rng(5)
    tg = np.flatnonzero(htil.ravel())
    cand = cand.ravel().copy()
    cand[tg] = rng.choice(np.flatnonzero(dsrc.ravel()), len(tg))
    dist = dist.ravel().copy()
    dist[tg] = rng.integers(0, 1 << 20, len(tg))
    nv = nvox.ravel().copy()
    nv[tg] = 125
    o.set_state(0, rgbt=rgbt, cand=cand.reshape(htil.shape), dist=dist.reshape(htil.shape),
                nvox=nv.reshape(htil.shape))
    t0 = time.perf_counter()
    o.reconstruct(0, vio.WEIGHTED)
    out["sd_l0_reconstruct_s"] = time.perf_counter() - t0
    out["sd_l0_hole_pixels"] = int(hole.sum())
    o.close()
    tiny = synth.tiny()
    o = vio.Oracle(tiny.occluded_input(), tiny.mask, levels=1, em_tol=-1.0, em_max_iters=10, seed=1)
    t0 = time.perf_counter()
    o.inpaint()
    out["tiny_inpaint_s"] = time.perf_counter() - t0
    o.close()
    print(json.dumps(out), flush=True)


def oracle_timing():
    import subprocess
    res = []
    for n in (1, os.cpu_count() or 1):
        env = dict(os.environ, OMP_NUM_THREADS=str(n))
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-timing-run"],
                           env=env, capture_output=True, text=True, check=True)
        res.append(json.loads(r.stdout.strip().splitlines()[-1]))
    print(json.dumps({"oracle_timing": res}), flush=True)


def percentile(xs, q):
    """Nearest-rank percentile (q in (0, 1]) of a list."""
    ys = sorted(xs)
    k = max(1, int(-(-q * len(ys) // 1)))  # ceil(q n)
    return ys[min(k, len(ys)) - 1]


def roofline_of(workload, pass_evals, pass_units, pass_ms, pass_launches, nominal_pass):
    """Roofline record of the propagation-pass kernel from a run's device
    counters and event times, and the counter record of the same kernel
    (profiles/k_pass_<workload>_counters.json) while its source matches."""
    avg_ms = pass_ms / pass_launches
    evals_per_launch = pass_evals / pass_launches
    targets_per_launch = pass_units / pass_launches
    bytes_per_launch = (BYTES_PER_EVAL * evals_per_launch
                        + BYTES_PER_TARGET_PASS * targets_per_launch)
    gbs = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    tops = OPS_PER_EVAL * evals_per_launch / (avg_ms * 1e-3) / 1e12
    # nominal evaluations of these launches (the onion peel's share, < 1 %,
    # is included)
    nominal_pass_per_launch = nominal_pass / pass_launches
    cnt = None
    path = counters_json(workload)
    if os.path.exists(path):
        cj = json.load(open(path))
        cc = cj.get("copy_calibration") or {}
        copy_gbs = (2.0 * cc["bytes"] / (cc["mean_us"] * 1e-6) / 1e9) if cc.get("mean_us") else None
        if cj.get("source_sha256") == kernel_source_hash():
            hbm_gbs = cj["hbm_bytes_per_launch"] / (cj["mean_launch_us"] * 1e-6) / 1e9
            cnt = {"hbm_bytes_per_launch": round(cj["hbm_bytes_per_launch"]),
                   "hbm_gbs": round(hbm_gbs, 1),
                   "achievable_copy_gbs": None if copy_gbs is None else round(copy_gbs, 1),
                   "hbm_frac_of_copy": None if copy_gbs is None else round(hbm_gbs / copy_gbs, 4),
                   "hbm_frac_of_peak": round(hbm_gbs / HBM_PEAK_GBS, 4),
                   "valu_busy": round(cj["valu_busy"], 4),
                   "profiled_mean_launch_us": round(cj["mean_launch_us"], 2),
                   "record": os.path.relpath(path, ROOT)}
    # the binding roof: the one the counters show nearer to saturation
    if cnt and cnt["hbm_frac_of_copy"] is not None and cnt["valu_busy"] > cnt["hbm_frac_of_copy"]:
        bound, achieved, peak, unit = "alu", tops, VALU_PEAK_TOPS, "TOP/s"
    else:
        bound, achieved, peak, unit = "hbm", gbs, HBM_PEAK_GBS, "GB/s"
    limiter = None
    if cnt:
        top = max(cnt["valu_busy"], cnt["hbm_frac_of_copy"] or 0.0)
        limiter = ("latency: neither the VALU nor HBM traffic reaches half of its roof"
                   if top < 0.5 else f"{bound} roof")
    return {
        "bound": bound, "achieved": round(achieved, 3), "peak": round(peak, 1), "unit": unit,
        "frac": round(achieved / peak, 4),
        "traffic": None if cnt is None else cnt["hbm_bytes_per_launch"],
        "kernel": "k_pass<false, false, *> (the exact-distance search pass on the levels with "
                  "more than 131072 targets: <false, false, false> with the random search "
                  "fused, every third pass; <false, false, true> the other passes, short "
                  "queues evaluated by lane groups; one template, timed together)",
        "avg_launch_ms": round(avg_ms, 5), "launches": pass_launches,
        "evals_per_launch": round(evals_per_launch, 1),
        "target_passes_per_launch": round(targets_per_launch, 1),
        "algorithmic_bytes_per_launch": round(bytes_per_launch),
        "algorithmic_gbs": round(gbs, 1), "algorithmic_frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
        "algorithmic_int_tops": round(tops, 3),
        "algorithmic_frac_of_valu_peak": round(tops / VALU_PEAK_TOPS, 4),
        "nominal_evals_per_launch": round(nominal_pass_per_launch, 1),
        "nominal_gather_gbs": round(BYTES_PER_EVAL * nominal_pass_per_launch
                                    / (avg_ms * 1e-3) / 1e9, 1),
        "counters": cnt, "limiter": limiter,
    }


def measure_plain(config, steps, warmup, em_iters, temporal=False, reduce_dims=0):
    """Whole inpaintings of one clip from inputs resident in HBM: timed
    steps, per-kind kernel time of one more step, and the roofline record
    (temporal: pyramids subsampled in time as well; reduce_dims: searches
    in the PCA-reduced patch space)."""
    import torch
    from paper_1503_05528_amd import vi
    clip, levels = make_clip(config)
    W, H, T = clip.shape
    video = torch.from_numpy(clip.occluded_input()).cuda()
    mask = torch.from_numpy(clip.mask).cuda()
    params = vi.default_params(levels=levels, em_tol=-1.0, em_max_iters=em_iters, seed=1,
                               temporal_subsample=1 if temporal else 0,
                               reduce_dims=reduce_dims)
    torch.cuda.synchronize()

    last = {}

    def one_step(profile=None):
        c0 = time.perf_counter()
        g = vi.Clip(video, mask, params=params)
        last["create_s"] = time.perf_counter() - c0
        if profile:
            g.profile(True, kinds=profile)
        out = g.inpaint()
        last["out"] = out
        rec = g.profile_read() if profile else []
        cnt = g.counters()
        g.close()
        return out, rec, cnt

    log(f"{config}: {warmup} warm-up and {steps} timed steps")
    for _ in range(warmup):
        one_step()
    torch.cuda.synchronize()
    lat = []
    recs = []
    nominal = effective = pass_evals = 0
    t0 = time.perf_counter()
    # inside the timed region only the search passes (the roofline's kernel)
    # are timed with events; every event pair costs the stream a few tens of
    # microseconds
    for _ in range(steps):
        s0 = time.perf_counter()
        out, rec, cnt = one_step(profile=("pass",))
        lat.append(time.perf_counter() - s0)
        recs += rec
        nominal += cnt["nominal_evals"]
        effective += cnt["effective_evals"]
        # the one-lane form's distances (small levels take the wide form)
        pass_evals += cnt["pass_evals"] - cnt["pass_wide_evals"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    def by_kind(rs):
        kinds = {}
        for kind, lvl, units, ms, nl in rs:
            d = kinds.setdefault(kind, {"launches": 0, "units": 0, "ms": 0.0})
            d["launches"] += nl
            d["units"] += units
            d["ms"] += ms
            d["targets_per_search"] = d.get("targets_per_search", 0) + units / max(nl, 1)
        return kinds
    kinds = by_kind(recs)
    # per kind and level: one more step, after the timed region, with every
    # kind timed
    _, all_recs, all_cnt = one_step(profile=tuple(vi.KERNEL_KINDS.values()))
    by_level = {}
    for kind, lvl, units, ms, nl in all_recs:
        key = f"{kind}@L{lvl}"
        by_level[key] = round(by_level.get(key, 0.0) + ms, 3)
    pas = kinds.get("pass", {"launches": 1, "units": 0, "ms": 1.0, "targets_per_search": 0})
    # the one-lane form's share of the passes' nominal evaluations: every
    # target-pass of a search has the same nominal count, and every search
    # one per target more (step 0), so the passes' nominal evaluations split
    # by target-passes
    ak = by_kind(all_recs)
    one, wide = ak.get("pass", {}), ak.get("pass_wide", {})
    u1, uw = one.get("units", 0), wide.get("units", 0)
    tps = one.get("targets_per_search", 0) + wide.get("targets_per_search", 0)
    nominal_one = (nominal - steps * tps) * (u1 / max(u1 + uw, 1))
    roof = roofline_of(config, pass_evals, pas["units"], pas["ms"], pas["launches"], nominal_one)
    pass_wide = None
    if wide:
        pass_wide = {
            "kernel": "k_pass_wide<64, false> (the same pass on small target lists, eight lanes per "
                      "distance)",
            "launches_per_step": wide["launches"], "ms_per_step": round(wide["ms"], 3),
            "avg_launch_ms": round(wide["ms"] / wide["launches"], 5),
            "target_passes_per_launch": round(uw / wide["launches"], 1),
            "evals_per_launch": round(all_cnt["pass_wide_evals"] / wide["launches"], 1),
            "levels": sorted({lvl for kind, lvl, _, _, _ in all_recs if kind == "pass_wide"}),
        }
    # mean |error| over the hole's colour channels against the clip's true video
    hole = torch.from_numpy(clip.mask).cuda().bool()
    err = (last["out"][hole].float() - torch.from_numpy(clip.video).cuda()[hole].float())
    hole_err = float(err.abs().mean())
    hole_psnr = float(10.0 * torch.log10(255.0 ** 2 / (err * err).mean()))
    return {
        "value": nominal / elapsed, "ms_per_step": 1000.0 * elapsed / steps,
        "clips_per_s": steps / elapsed, "steps": steps, "warmup": warmup,
        "workload": f"{config} plain run {W}x{H}x{T}, {levels}-level pyramid"
                    f"{' subsampled in time as well' if temporal else ''}, 5x5x5 patches"
                    f"{f' compared in a {reduce_dims}-dimensional PCA space' if reduce_dims else ''}"
                    f", {em_iters} EM iterations per level, one clip per step",
        "hole_mean_abs_error": hole_err,
        "hole_psnr_db": hole_psnr,
        "create_ms": 1000 * last["create_s"],
        "latency_p50_ms": 1000 * percentile(lat, 0.5),
        "latency_p99_ms": 1000 * percentile(lat, 0.99),
        "latency_samples": len(lat),
        "effective_evals_per_s": effective / elapsed,
        "kernel_ms_per_step": {k: round(v["ms"], 3) for k, v in by_kind(all_recs).items()},
        "kernel_ms_per_step_by_level": by_level,
        "roofline": roof,
        "pass_wide": pass_wide,
        "clip": (clip, levels),
    }


def main():
    a = parse()
    if a.oracle_timing_run:
        oracle_timing_run()
        return
    if a.oracle_timing:
        oracle_timing()
        return
    if a.cpu_sample_run:
        cpu_sample_run(a.cpu_sample_run[0], int(a.cpu_sample_run[1]))
        return
    if a.summarize_counters:
        print(json.dumps(summarize_counters(a.summarize_counters), indent=1))
        return
    if a.assemble_counters:
        print(json.dumps(assemble_counters(*a.assemble_counters, a.config), indent=1))
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported "
              "(the per-clip path and its batching are single-GPU)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1503_05528_amd import vi

    if a.copy_calibration:
        n = 1 << 30
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "launches": 3}))
        return

    vi.lib()
    if a.appb_only:
        print(json.dumps(measure_appb()), flush=True)
        return
    if a.served_sweep:
        rates = [float(r) for r in a.served_sweep.split(",")]
        print(json.dumps(served_sweep(rates, a.served_jobs, a.em_iters)), flush=True)
        return
    m = measure_plain(a.config, a.steps, a.warmup, a.em_iters, reduce_dims=a.reduce_dims)
    clip, levels = m.pop("clip")
    line = {
        "metric": "NNF patch-distance evals/s (nominal)",
        "value": m["value"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": m["workload"], "global_batch": 1},
        "clips_per_s": m["clips_per_s"],
        "latency_p50_ms": m["latency_p50_ms"],
        "latency_p99_ms": m["latency_p99_ms"],
        "latency_samples": m["latency_samples"],
        "effective_evals_per_s": m["effective_evals_per_s"],
        "hole_mean_abs_error": m["hole_mean_abs_error"],
        "hole_psnr_db": m["hole_psnr_db"],
        "kernel_ms_per_step": m["kernel_ms_per_step"],
        "kernel_ms_per_step_by_level": m["kernel_ms_per_step_by_level"],
        "roofline": m["roofline"],
        "pass_wide": m["pass_wide"],
        "cpu_baseline": None,
    }
    sd_clip = None
    if not a.no_sd and a.config != "sd":
        s = measure_plain("sd", a.sd_steps, 1, a.em_iters)
        sd_clip = s.pop("clip")
        line["sd"] = {k: s[k] for k in ("workload", "value", "ms_per_step", "clips_per_s",
                                        "latency_p50_ms", "effective_evals_per_s",
                                        "kernel_ms_per_step")}
        line["sd"]["roofline"] = {k: s["roofline"][k] for k in
                                  ("bound", "achieved", "peak", "unit", "frac", "traffic",
                                   "avg_launch_ms", "algorithmic_frac_of_hbm_peak", "counters")}
        line["sd"]["pass_wide"] = s["pass_wide"]
        line["sd"]["ms_per_step_service"] = s["latency_p50_ms"]
    elif a.config == "sd":
        sd_clip = (clip, levels)
    if not a.no_sd:
        # the SD clip with temporally subsampled pyramids (Sec. 3.6)
        s = measure_plain("sd", a.sd_steps, 1, a.em_iters, temporal=True)
        s.pop("clip")
        line["sd_temporal"] = {k: s[k] for k in ("workload", "value", "ms_per_step",
                                                 "clips_per_s", "kernel_ms_per_step")}
    if not a.no_realign:
        log("realignment: shaking-camera clip")
        line["realign"] = measure_realign()
    if not a.no_reduced:
        # the reduced patch space (Sec. 5) on the headline clip
        r = measure_plain(a.config, 2, 1, a.em_iters, reduce_dims=16)
        r.pop("clip")
        line["reduced"] = {k: r[k] for k in ("workload", "value", "ms_per_step", "create_ms",
                                             "kernel_ms_per_step", "hole_mean_abs_error",
                                             "hole_psnr_db")}
        line["reduced"]["exact_hole_mean_abs_error"] = m["hole_mean_abs_error"]
        line["reduced"]["exact_ms_per_step"] = m["ms_per_step"]
    if not a.no_image:
        log("images: 5x5x1 patches")
        line["image"] = measure_image()
    if not a.no_appb:
        log("App. B: random patches against the constant patch")
        line["appb"] = measure_appb()
    if not a.no_batched or not a.no_served:
        bclips = gen_batch_clips(a.batch_clips)
        bres, service = batched_vs_serial(bclips, a.em_iters)
        if not a.no_batched:
            line["batched"] = bres
        if not a.no_served:
            log(f"served: {a.served_seconds} s Poisson trace")
            svc = {i: service[i] for i in range(len(bclips))}
            if sd_clip is None:
                sd_clip = make_clip("sd")
            svc[-1] = (line["sd"]["ms_per_step_service"] / 1000.0 if "sd" in line
                       else m["latency_p50_ms"] / 1000.0)
            c, L = sd_clip
            line["served"] = served(bclips, (c.occluded_input(), c.mask, L),
                                    a.served_seconds, a.served_rate, a.em_iters, svc)
    if not a.no_cpu_baseline:
        log("cpu baseline: oracle search on a sample of the finest level")
        line["cpu_baseline"] = cpu_baseline(a.config, a.cpu_frames, a.cpu_frames_1core)
        if "realign" in line:
            line["realign"]["cpu_baseline"] = realign_cpu_baseline()
        if "appb" in line:
            line["appb"]["cpu_baseline"] = appb_cpu_baseline()
        if "image" in line:
            line["image"]["cpu_baseline"] = image_cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
