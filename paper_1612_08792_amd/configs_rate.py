"""Per-iteration rates of the EM on the benchmark workloads, paper T mode (a
fixed number of iterations, Algorithm 1): 481x321 (K 400, T = 10), 1920x1080
(K 2000, T = 20), the uneven batch of 64 images (T = 15) and the 4K batch
(32 x 3840x2160, K 10000, T = 10).  Each workload is autotuned (kind, rows per
chunk and waves per cell of the statistics pass, lanes per superpixel of the
gather, per-pass or persistent launches), then timed in three launch forms --
per-pass launches, graph replay of the T passes, and one persistent
cooperative launch of the T passes (the fastest counts):

  * Mpix/s per iteration = total pixels x iterations / wall time of the
    iterations (E-step, statistics, gather, LL and stop rule; inputs resident);
  * the E-step alone (one more, eager run): HIP-event time of its launches on
    the launch stream, Gpx/s per pass and TFLOP/s of the 54 algorithmic flops per (pixel,
    candidate) pair, against the 157.3 TFLOP/s FP32 vector peak (and the 78.6
    TFLOP/s single-rate issue of FMAs that read a scalar register).

    python -m paper_1612_08792_amd.configs_rate [--configs 1,2,3,5] [--repeats 5]

With workload 1 it also times Algorithm 1 end to end (seeds, T = 10, labels,
connectivity) per 481x321 image, alone and in a batch of 64.  Prints one JSON
line per measurement and a markdown table."""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from paper_1612_08792_amd.gmmsp import GMMSP  # noqa: E402

PEAK_FP32 = 157.3   # TFLOP/s, FP32 vector (256 CU x 4 SIMD x 32 x 2 x 2.4 GHz)
PEAK_SINGLE = 78.6  # TFLOP/s, a wave64 FMA every 4 cycles per SIMD
FLOPS_PER_PAIR = 54.0


def workload(c: int, dev):
    if c == 1:
        return "481x321, K 400, T 10", [synth.config1_image(dev)], 10
    if c == 2:
        return "1920x1080, K 2000, T 20", [synth.config2_image(dev)], 20
    if c == 3:
        return "64 uneven images, T 15", synth.config3_batch(dev), 15
    return "32 x 3840x2160, K 10000, T 10", synth.config5_batch(dev), 10


def end_to_end(dev, repeats: int):
    """Algorithm 1 on 481x321 images (K 400, T = 10): seeds, ten iterations,
    labels and the connectivity step, wall time per image, one image alone and
    in a batch of 64 images of the same law."""
    for n in (1, 64):
        ims = [synth.config4_image(20000 + i, dev) for i in range(n)]
        lab = synth.pack_batch(ims).contiguous()
        m = GMMSP([(im.W, im.H) for im in ims], K=400, device=dev)
        m.autotune(lab, passes=3, cache=None)
        m.set_graph_passes(10)
        ts = []
        for r in range(repeats + 1):
            torch.cuda.synchronize(dev)
            t0 = time.perf_counter()
            m.init_seeds(lab)
            m.em_iterate(lab, 10)
            labels, _ = m.label(lab, want_ll=False)
            m.connectivity(lab, labels)
            torch.cuda.synchronize(dev)
            if r:                                    # the first run captures the graph
                ts.append(time.perf_counter() - t0)
        t = float(np.median(ts))
        print(json.dumps({"algorithm1_481x321_T10": n, "ms_per_image": round(1e3 * t / n, 4),
                          "mpix_per_s": round(m.n_pixels / t / 1e6, 1)}), flush=True)
        m.close()


def measure(c: int, dev, repeats: int = 5) -> dict:
    """Per-iteration rates of workload c: autotuned schedule, wall time of T
    iterations with per-pass launches, graph replay and the persistent launch
    (median of `repeats`), and the E-step alone from HIP events in one more
    run of per-pass launches."""
    name, ims, T = workload(c, dev)
    lab = synth.pack_batch(ims).contiguous()
    m = GMMSP([(im.W, im.H) for im in ims], K=[im.K for im in ims], device=dev)
    m.autotune(lab, passes=3, cache=None)
    sched = m.schedule()

    def wall(graph: int, persistent: bool = False) -> float:
        m.set_graph_passes(graph)
        m.set_persistent(persistent)
        m.init_seeds(lab)
        m.em_iterate(lab, T)                        # warm-up (graph capture)
        walls = []
        for _ in range(repeats):
            m.init_seeds(lab)
            torch.cuda.synchronize(dev)
            t0 = time.perf_counter()
            m.em_iterate(lab, T)
            torch.cuda.synchronize(dev)
            walls.append(time.perf_counter() - t0)
        return float(np.median(walls))

    t_eager, t_graph = wall(0), wall(T)
    # the persistent launch runs the slot-lane pass (kind 1): timed with it
    has_slots = m.cov_mode == 0 and m.get_slot_rows() > 0
    t_pers = float("inf")
    if has_slots:
        m.set_estep_kernel(1)
        t_pers = wall(0, True)
        m.set_estep_kernel(sched["estep_kernel"])
    forms = {"per_pass": t_eager, "graph": t_graph, "persistent": t_pers}
    best_form = min(forms, key=forms.get)
    t = forms[best_form]
    m.set_persistent(bool(sched["persistent"]))
    # the E-step alone: an eager run with events around each launch (the
    # library replays no graph while it profiles)
    m.set_graph_passes(0)
    m.profile(True)
    m.profile_read(True)
    m.init_seeds(lab)
    m.em_iterate(lab, T)
    p = m.profile_read(True)
    m.profile(False)
    est = p["estep_ms"] / p["launches"]
    tflops = p["pair_evals"] * FLOPS_PER_PAIR / (p["estep_ms"] / 1e3) / 1e12
    r = dict(config=c, workload=name, images=len(ims), pixels=m.n_pixels, T=T,
             schedule=sched, statistics_pass_ms=m.tune_ms,
             gather_ms={k: round(v, 4) for k, v in m.tune_gather_ms.items()},
             mpix_per_s_per_iteration=round(m.n_pixels * T / t / 1e6, 1),
             ms_per_iteration=round(1e3 * t / T, 4),
             ms_per_iteration_eager=round(1e3 * t_eager / T, 4),
             ms_per_iteration_graph=round(1e3 * t_graph / T, 4),
             ms_per_iteration_persistent=(round(1e3 * t_pers / T, 4) if has_slots else None),
             fastest_form=best_form, launch_form_ms=m.tune_persistent_ms,
             estep_ms_per_launch=round(est, 4),
             estep_gpx_per_s=round(p["pixel_evals"] / (p["estep_ms"] / 1e3) / 1e9, 2),
             pairs_per_pixel=round(p["pair_evals"] / p["pixel_evals"], 3),
             estep_tflops=round(tflops, 2), frac_of_157_3=round(tflops / PEAK_FP32, 3),
             frac_of_78_6=round(tflops / PEAK_SINGLE, 3))
    m.close()
    del m, lab, ims
    torch.cuda.empty_cache()
    return r


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--configs", type=str, default="1,2,3,5")
    ap.add_argument("--repeats", type=int, default=5)
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    rows = []
    for c in (int(x) for x in args.configs.split(",")):
        r = measure(c, dev, args.repeats)
        print(json.dumps(r), flush=True)
        rows.append(r)
    if 1 in [int(x) for x in args.configs.split(",")]:
        end_to_end(dev, args.repeats)
    print("| workload | Mpix/s per iteration | ms per iteration (per-pass / graph / persistent) | "
          "E-step us | E-step Gpx/s | TFLOP/s | of 157.3 | schedule (kind, rows, waves per cell, "
          "gather lanes, persistent) |")
    print("|---|---:|---|---:|---:|---:|---:|---|")
    for r in rows:
        sc = r["schedule"]
        pers = r["ms_per_iteration_persistent"]
        print(f"| {r['workload']} | {r['mpix_per_s_per_iteration']:.0f} | "
              f"{r['ms_per_iteration_eager']:.4f} / {r['ms_per_iteration_graph']:.4f} / "
              f"{'-' if pers is None else f'{pers:.4f}'} | "
              f"{1e3 * r['estep_ms_per_launch']:.0f} | {r['estep_gpx_per_s']:.1f} | "
              f"{r['estep_tflops']:.1f} | {r['frac_of_157_3']:.2f} | "
              f"{sc['estep_kernel']}, {sc['rows_per_chunk']}, {sc['waves_per_cell']}, "
              f"{sc['gather_lanes']}, {sc['persistent']} |")


if __name__ == "__main__":
    main()
