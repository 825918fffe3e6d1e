"""Launch the fused iteration kernel back-to-back on a fixed workload and
report its mean duration (HIP events on the library stream) with the derived
segment x edge test rate.  Meant to run under rocprofv3:

  rocprofv3 --kernel-trace --stats -d OUT -- python -m paper_2308_10169_amd.profile_kernel
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

PEAK_FP32 = 157.3e12
F_TEST = 10.0


def workload(name, instances):
    from paper_2308_10169_amd import inputs as I
    if name == "batch":
        specs, sws = [], []
        for i in range(instances):
            m, shape = I.batch_instance(i, 0)
            sws.append(I.dynamic_swarm(m.scale, seed=0, instance=i, **shape))
            specs.append(m)
        return specs, sws
    if name == "stress":
        spec = I.stress_map(0)
        sw = I.SwarmSpec(8, 4096, 64, 200, I.HYPER8PATH, alpha=30.0, beta=4, seed=0,
                         hsef_every=10)
        return [spec], [sw]
    if name == "paper":
        spec = I.dynamic_map(0)
        return [spec], [I.dynamic_swarm(spec.scale, seed=0)]
    raise ValueError(name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="batch", choices=["batch", "stress", "paper"])
    ap.add_argument("--instances", type=int, default=1024)
    ap.add_argument("--tune", default="16,64", help="K,block_threads or 'auto'")
    ap.add_argument("--launches", type=int, default=20)
    ap.add_argument("--warmup-launches", type=int, default=20)
    ap.add_argument("--frames-first", type=int, default=1,
                    help="frames planned before the warm-up launches (the benchmark's state)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="also run a plain device-to-device copy of this many MiB (counter scale)")
    args = ap.parse_args()
    from paper_2308_10169_amd import sepso
    specs, sws = workload(args.workload, args.instances)
    tune = None if args.tune == "auto" else tuple(int(v) for v in args.tune.split(","))
    bp = sepso.BatchPlanner(specs, sws, tune=tune)
    if tune is None:
        tune = bp.autotune()
    tests, elems = bp.work()
    if args.frames_first > 0:
        bp.plan(args.frames_first)
    if args.warmup_launches > 0:
        bp.profile_step(args.warmup_launches)  # clocks settle before the measured launches
    ms = bp.profile_step(args.launches)
    rate = tests / (ms * 1e-3)
    print(json.dumps(dict(workload=args.workload, instances=len(specs), tune=tune,
                          launches=args.launches, ms_per_launch=ms, tests_per_launch=tests,
                          elems_per_launch=elems, tests_per_s=rate,
                          tflops_alg=F_TEST * rate / 1e12, frac_peak=F_TEST * rate / PEAK_FP32)),
          flush=True)
    bp.close()
    if args.copy_mb > 0:
        import torch
        n = args.copy_mb << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_bytes=n, copies=3)), flush=True)


if __name__ == "__main__":
    main()
