"""Benchmark of the fused radiative-transfer step on one MI355X.

Workload: 3D periodic box 128^3, 80 directions (level-symmetric S8), FP64
intensities, rho lognormal(1), T lognormal(0.3), v Gaussian (rms 0.02 c per
component), sigma_a = 0.1 rho, sigma_s = rho, dt at Courant 0.4; the same box
is also timed with FP32 intensities and FP64 temperature solve.  A step is
one fused launch doing transport, velocity estimate, absorption, scattering
and quadrature for every cell and angle, plus the small reduction of the
domain totals.  Inputs are resident in device memory before timing starts.

Prints one JSON line (rank 0): the FP64 throughput in cell-angle updates/s,
the roofline of the fused kernel (algorithmic bytes per launch over the mean
launch time from HIP events recorded around each launch on its stream), the
FP32-mixed throughput, and the CPU oracle's rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-angle updates/s, FP64 vs FP32-mixed; p50/p99 latency of served solves"
HBM_PEAK_GBS = 8000.0
FIELD_BYTES_PER_CELL = 232  # 14 FP64 per-cell reads + 15 FP64 per-cell writes


def algorithmic_bytes_per_cell(nang: int, sbytes: int) -> int:
    """I read once and written once per angle, plus the per-cell fields."""
    return 2 * sbytes * nang + FIELD_BYTES_PER_CELL


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch measured with rocprofv3 counters, if a summary for
    this kernel and workload is committed under profiles/."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
        return d.get("bytes_per_launch")
    except Exception:
        return None


def run_gpu(wl, precision: str, steps: int, warmup: int, second_order: bool = False):
    import torch

    import workloads as W
    from paper_1403_6126_amd import rt
    from paper_1403_6126_amd.solver import Solver, quadrature_for

    mu, w = quadrature_for(wl.quad)
    T = torch.as_tensor(wl.T).cuda()
    I0 = W.equilibrium_intensity(T, len(w), xp=torch)  # (nang, ncell), expanded view
    s = Solver(wl, precision=precision, mu=mu, w=w, I0=I0, second_order=second_order)
    del I0
    info = rt.rt_get_info(s.ctx)
    stream = torch.cuda.current_stream().cuda_stream
    if warmup:
        rt.rt_step(s.ctx, wl.dt, warmup, s.fields, s.out, stream)
    torch.cuda.synchronize()
    rt.rt_profile_read(s.ctx)  # discard
    rt.rt_profile_enable(s.ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rt.rt_step(s.ctx, wl.dt, steps, s.fields, s.out, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kms, nl = rt.rt_profile_read(s.ctx)
    rt.rt_profile_enable(s.ctx, False)
    status = s.status()
    totals = s.totals.cpu().tolist()
    s.close()
    if status != 0:
        raise RuntimeError(f"device status {status} after the timed steps")
    wall = t1 - t0
    upd = wl.ncell * info.nang * steps
    kavg = kms / max(nl, 1) / 1e3
    bpl = algorithmic_bytes_per_cell(info.nang, info.storage_bytes) * wl.ncell
    return dict(value=upd / wall, ms_per_step=wall / steps * 1e3, kernel_ms=kavg * 1e3,
                launches=nl, bytes_per_launch=bpl, achieved_gbs=bpl / kavg / 1e9,
                nang=info.nang, storage_bytes=info.storage_bytes, totals=totals,
                grid_blocks=info.grid_blocks, block_threads=info.block_threads)


def cpu_baseline(wl, budget_s: float = 12.0, batch: int = 65536, seed: int = 0,
                 threads: int = 0):
    """The CPU oracle (as it stands) on a bounded sample of the same workload:
    one step evaluated on batches of random cells of the 128^3 box until the
    time budget is spent, on all host threads or on `threads` of them."""
    import numpy as np

    import oracle

    if threads > 0:
        oracle.set_threads(threads)
    prob = oracle.Problem(wl)
    I = wl.init(prob.mu)
    rng = np.random.default_rng(seed)
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        cells = np.sort(rng.choice(wl.ncell, batch, replace=False))
        oracle.step_cells(prob, I, wl.T, cells)
        done += len(cells)
    el = time.perf_counter() - t0
    return dict(value=done * prob.nang / el, unit="cell-angle updates/s", cores=oracle.threads(),
                kind="oracle",
                sample=f"one step at {done} randomly sampled cells of the 128^3 S8 FP64 box "
                       f"(batches of {batch}; each batch also takes the moments of all cells), "
                       f"{el:.1f} s")


SERVE_DEFAULTS = dict(pool_bytes=96 << 30, max_active=1024, packed_cells=4096,
                      chunk_work=400_000_000, large_work=40_000_000)


def serving(count: int, load: float, warm: int, seed: int = 4, fifo: bool = True):
    """The serving stream: `count` requests of the mixed-size trace (1D/2D/3D
    grids of 64 to 128^3 cells log-uniform, 16-288 directions, 10-200 steps,
    FP32-mixed, Poisson arrivals).  The batched capacity is measured first in
    a closed loop over the first `warm` requests; arrivals are then scaled so
    that the offered load is `load` times that capacity, and the same trace
    runs through the server and through the plain one-at-a-time path.  The
    capacity run takes the whole trace by default: a prefix of a heavy-tailed
    mix need not carry its mean cost."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1403_6126_amd import serve

    def say(msg):
        print(f"bench: serving {msg}", file=sys.stderr, flush=True)

    reqs = W.config4_requests(count, seed=seed)
    wls = [W.request_workload(r, precision="mixed") for r in reqs]
    work = np.array([wl.ncell * wl.nsteps * _nang(r["quad"]) for wl, r in zip(wls, reqs)],
                    dtype=np.float64)
    say(f"{count} requests generated")
    warm = warm if 0 < warm < count else count
    cap = serve.run_batched(wls[:warm], [0.0] * warm, progress=say, **SERVE_DEFAULTS)
    rate = load * cap["throughput"] / work.mean()          # requests per second
    arrivals = np.cumsum([r["gap"] for r in reqs]) / rate
    arrivals -= arrivals[0]
    print(f"bench: serving capacity {cap['throughput']:.3g} updates/s, offered "
          f"{rate:.3g} req/s over {arrivals[-1]:.1f} s", file=sys.stderr, flush=True)
    b = serve.run_batched(wls, arrivals, progress=say, **SERVE_DEFAULTS)
    print(f"bench: served p50 {b['latency_p50_s']*1e3:.1f} ms p99 {b['latency_p99_s']*1e3:.1f} ms "
          f"{b['throughput']:.3g} updates/s", file=sys.stderr, flush=True)
    torch.cuda.empty_cache()
    f = None
    if fifo:
        f = serve.run_fifo(wls, arrivals, progress=say)
        print(f"bench: fifo p50 {f['latency_p50_s']*1e3:.1f} ms p99 {f['latency_p99_s']*1e3:.1f} ms "
              f"{f['throughput']:.3g} updates/s", file=sys.stderr, flush=True)
    return dict(requests=count, load=load, closed_loop_capacity=cap["throughput"],
                offered_req_per_s=rate, mean_updates_per_request=float(work.mean()),
                batched=b, fifo=f, server=SERVE_DEFAULTS,
                latency="submission to results in host memory")


def _nang(quad):
    return quad[1] if quad[0] == "gl" else quad[1] * (quad[1] + 2)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--nper", type=int, default=128, help="cells per axis (128 = full workload)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the CPU-baseline leg (0: all host threads)")
    ap.add_argument("--only-cpu", action="store_true",
                    help="run the CPU-baseline leg alone (no GPU) and print its JSON")
    ap.add_argument("--only", choices=["fp64", "mixed"], default=None,
                    help="profiling: run one precision only and print its timing")
    ap.add_argument("--second-order", action="store_true",
                    help="with --only: time the step with the absorption system solved twice "
                         "(the thread-per-cell kernel)")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="requests of the serving trace (0: skip; 2000 = the full stream)")
    ap.add_argument("--serve-load", type=float, default=0.8)
    ap.add_argument("--serve-warm", type=int, default=0,
                    help="requests of the closed-loop capacity run (0: the whole trace)")
    ap.add_argument("--only-serve", action="store_true")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="profiling: time a plain device-to-device copy of this many GiB "
                         "(counter calibration) and exit")
    args = ap.parse_args()
    if args.second_order and not args.only:
        ap.error("--second-order goes with --only")
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the library "
              "has no multi-GPU path (the domain decomposition it would use is a design, "
              "not code)", file=sys.stderr)
        sys.exit(2)
    if args.only_cpu:
        import workloads as W
        print(json.dumps(cpu_baseline(W.config2(nper=args.nper), args.cpu_budget,
                                      threads=args.cpu_threads)), flush=True)
        return

    import torch

    import workloads as W

    assert torch.cuda.is_available(), "no GPU visible"
    torch.cuda.set_device(0)
    if args.copy_probe > 0:
        # a plain device-to-device copy: the counter calibration, and the
        # measured bandwidth the step kernels can be set against
        n = int(args.copy_probe * (1 << 30)) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        print(json.dumps({"copy_probe_bytes_each_way": 8 * n, "launches": args.steps,
                          "ms_per_copy": ms, "read_plus_write_gbs": 2 * 8 * n / ms / 1e6}))
        return
    if args.only_serve:
        print(json.dumps(serving(args.serve_requests, args.serve_load, args.serve_warm)),
              flush=True)
        return
    wl = W.config2(nper=args.nper)
    wname = f"box3d_{args.nper}cube_S8"
    print(f"bench: {wname} fp64 warmup={args.warmup} steps={args.steps}", file=sys.stderr,
          flush=True)
    if args.only:
        r = run_gpu(wl, args.only, args.steps, args.warmup, second_order=args.second_order)
        print(json.dumps({"precision": args.only, "second_order": args.second_order,
                          "kernel_ms": r["kernel_ms"], "value": r["value"],
                          "achieved_gbs": r["achieved_gbs"],
                          "bytes_per_launch": r["bytes_per_launch"],
                          "grid_blocks": r["grid_blocks"],
                          "block_threads": r["block_threads"]}), flush=True)
        return
    r64 = run_gpu(wl, "fp64", args.steps, args.warmup)
    print(f"bench: fp64 {r64['value']:.4g} cell-angle/s, kernel {r64['kernel_ms']:.3f} ms",
          file=sys.stderr, flush=True)
    mixed = None
    if not args.no_mixed:
        rmx = run_gpu(wl, "mixed", args.steps, args.warmup)
        print(f"bench: mixed {rmx['value']:.4g} cell-angle/s, kernel {rmx['kernel_ms']:.3f} ms",
              file=sys.stderr, flush=True)
        mixed = dict(value=rmx["value"], ms_per_step=rmx["ms_per_step"], dtype="f32 (I), f64 (T)",
                     roofline=dict(bound="hbm", achieved=rmx["achieved_gbs"], peak=HBM_PEAK_GBS,
                                   unit="GB/s", frac=rmx["achieved_gbs"] / HBM_PEAK_GBS,
                                   traffic=load_traffic("k_step3_mixed", wname),
                                   kernel="rtk::k_step3<float, float, 10, 1, true, true>",
                                   kernel_ms=rmx["kernel_ms"],
                                   bytes_per_launch=rmx["bytes_per_launch"]))
    srv = None
    if args.serve_requests > 0:
        import torch
        torch.cuda.empty_cache()
        srv = serving(args.serve_requests, args.serve_load, args.serve_warm)
    cpu = None
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(wl, args.cpu_budget, threads=args.cpu_threads)
    line = {
        "metric": METRIC,
        "value": r64["value"],
        "unit": "cell-angle updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded generator, no dataset)",
        "config": {"workload": f"{wname} periodic, FP64 fused step (transport + velocity "
                               "estimate + absorption + scattering + quadrature)",
                   "grid": [args.nper] * 3, "angles": r64["nang"], "courant": 0.4,
                   "kappa_a": 0.1, "kappa_s": 1.0, "launch": {"blocks": r64["grid_blocks"],
                                                              "threads": r64["block_threads"]}},
        "roofline": {"bound": "hbm", "achieved": r64["achieved_gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": r64["achieved_gbs"] / HBM_PEAK_GBS,
                     "traffic": load_traffic("k_step3_fp64", wname),
                     "kernel": "rtk::k_step3<double, double, 10, 1, true, true>",
                     "kernel_ms": r64["kernel_ms"], "bytes_per_launch": r64["bytes_per_launch"]},
        "fp32_mixed": mixed,
        "serving": srv,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
