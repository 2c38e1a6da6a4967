"""Benchmark of the inpainting hot path on one MI355X.

A step is one complete inpainting of the SD clip (854x480 px x 100 frames,
4-level pyramid, 5x5x5 patches, 20 EM iterations per level): context
creation (pyramids, texture features, sets), onion-peel initialisation, the
EM loop of every level (ANN search + weighted reconstruction), level
transitions and the final best-patch reconstruction, from the input video
resident in HBM to the output video in HBM.

Prints one JSON line.  `value` is nominal NNF patch-distance evaluations per
second over the timed steps (the nominal count of a search is |H~| x (1 + sum
over iterations of 6 n_jf + [radius >= 1]) and does not depend on how many
candidates an implementation skips).  The roofline object covers the
propagation-pass kernel, timed with HIP events on the context's stream over
the timed steps; the CPU baseline is the oracle's search at level 1 of the
same clip on the host cores.
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
BYTES_PER_EVAL = 625  # 125 voxels x 5 uint8 channels of the candidate patch


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="sd", choices=["sd", "hd", "tiny"])
    ap.add_argument("--em-iters", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-level", type=int, default=1)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    return ap.parse_args()


def make_clip(name):
    from paper_1503_05528_amd import synth
    if name == "sd":
        return synth.sd(), 4
    if name == "hd":
        return synth.hd(), 5
    return synth.tiny(), 1


def cpu_baseline(clip, levels, em_iters, level):
    """The oracle, as it stands, on a bounded sample of the workload: one ANN
    search at a coarser level of the same clip, on all host threads."""
    from oracle import vio
    o = vio.Oracle(clip.occluded_input(), clip.mask, levels=levels, em_tol=-1.0,
                   em_max_iters=em_iters, seed=1)
    (W, H, T), (nH, nS, nD) = o.info(level)
    per = 1
    p = o.params
    rmax = max(W, H, T)
    for k in range(1, p.pm_iters + 1):
        r = float(rmax)
        for _ in range(k):
            r *= p.rho
        per += 6 * p.n_jf + (1 if int(r // 1) >= 1 else 0)
    t0 = time.perf_counter()
    o.nnf_search(level, 0)
    dt = time.perf_counter() - t0
    evals = per * nS
    return {"value": evals / dt, "unit": "evals/s", "cores": vio.num_threads(),
            "kind": "oracle",
            "sample": f"one vio_nnf_search at pyramid level {level} of the same clip "
                      f"({W}x{H}x{T}, {nS} targets, {evals} nominal evals, {dt:.1f} s)"}


def main():
    a = parse()
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
    clip, levels = make_clip(a.config)
    W, H, T = clip.shape
    video = torch.from_numpy(clip.occluded_input()).cuda()
    mask = torch.from_numpy(clip.mask).cuda()
    params = vi.default_params(levels=levels, em_tol=-1.0, em_max_iters=a.em_iters, seed=1)
    torch.cuda.synchronize()

    def one_step(profile=False):
        g = vi.Clip(video, mask, params=params)
        if profile:
            g.profile(True)
        out = g.inpaint()
        rec = g.profile_read() if profile else []
        cnt = g.counters()
        g.close()
        return out, rec, cnt

    for _ in range(a.warmup):
        one_step()
    torch.cuda.synchronize()
    lat = []
    recs = []
    nominal = effective = 0
    t0 = time.perf_counter()
    for _ in range(a.steps):
        s0 = time.perf_counter()
        out, rec, cnt = one_step(profile=True)
        lat.append(time.perf_counter() - s0)
        recs += rec
        nominal += cnt["nominal_evals"]
        effective += cnt["effective_evals"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1000.0 * elapsed / a.steps

    kinds = {}
    for kind, lvl, units, ms in recs:
        d = kinds.setdefault(kind, {"launches": 0, "units": 0, "ms": 0.0})
        d["launches"] += 1
        d["units"] += units
        d["ms"] += ms
    by_level = {}
    for kind, lvl, units, ms in recs:
        key = f"{kind}@L{lvl}"
        by_level[key] = round(by_level.get(key, 0.0) + ms / a.steps, 3)
    pas = kinds.get("pass", {"launches": 1, "units": 0, "ms": 1.0})
    avg_ms = pas["ms"] / pas["launches"]
    bytes_per_launch = BYTES_PER_EVAL * pas["units"] / pas["launches"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    roofline = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
        "kernel": "k_pass (propagation + fused random search)",
        "avg_launch_ms": round(avg_ms, 5), "launches": pas["launches"],
        "evals_per_launch": round(pas["units"] / pas["launches"], 1),
    }
    line = {
        "metric": "NNF patch-distance evals/s (nominal)",
        "value": nominal / elapsed,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"{a.config} plain run {W}x{H}x{T}, {levels}-level pyramid, "
                               f"5x5x5 patches, {a.em_iters} EM iterations per level, one clip "
                               "per step",
                   "global_batch": 1},
        "clips_per_s": a.steps / elapsed,
        "latency_p50_ms": 1000 * statistics.median(lat),
        "latency_p99_ms": 1000 * max(lat),
        "effective_evals_per_s": effective / elapsed,
        "kernel_ms_per_step": {k: round(v["ms"] / a.steps, 3) for k, v in kinds.items()},
        "kernel_ms_per_step_by_level": by_level,
        "roofline": roofline,
        "cpu_baseline": None,
    }
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(clip, levels, a.em_iters, a.cpu_level)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
