"""Benchmark of the fused radiative-transfer step on one MI355X.

Workload: 3D periodic box 128^3, 80 directions (level-symmetric S8), FP64
intensities, rho lognormal(1), T lognormal(0.3), v Gaussian (rms 0.02 c per
component), sigma_a = 0.1 rho, sigma_s = rho, dt at Courant 0.4; the same box
is also timed with FP32 intensities and FP64 temperature solve.  A step is
one fused launch doing transport, velocity estimate, absorption, scattering
and quadrature for every cell and angle, plus the small reduction of the
domain totals.  Inputs are resident in device memory before timing starts.

Prints one JSON line (rank 0): the FP64 throughput in cell-angle updates/s,
the HBM roofline of the fused kernel (algorithmic bytes per launch over the
mean launch time from HIP events recorded around each launch on its stream)
and its VALU-issue roofline (algorithmic operations over the same time), the
FP32-mixed throughput on the same box and on the 256^3 shadow and
512x512x256 diffusion boxes, the serving trace against the plain path, and
the CPU oracle's steps-only rate on the host.
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
# VALU issue peak of one MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane
# operations per second (one FP64, or unpacked FP32, operation per lane and
# cycle; an FMA counts as one operation).
VALU_ISSUE_PEAK = 256 * 4 * 16 * 2.4e9
# Algorithmic VALU operations of one 3D cell-angle update, counted from the
# method with every interface value formed once (shared by its two cells)
# and the per-cell work amortised over the angles:
#   transport (Section 4.2), per angle: IV = n.W (3), I~ = I - IV/C (1); per
#     axis: the two differences (2), the two van Leer slopes (5 each: product,
#     sum, reciprocal, quotient, select), the upwind I~ and IV face values
#     (3), the alpha blend (3), the flux C x + IV* (1), the increment (2):
#     4 + 3 x 21 = 67;
#   source (Sections 4.3-4.5), per angle: n.u (3), D and the scattering
#     diagonal (2), their reciprocals (4), e, g, b, c (5), the routing (2),
#     the 22 sums of the reduced systems with their 7 shared products (29),
#     the new intensity (6), the 10 moments (10): 61.
ALG_OPS_PER_CELL_ANGLE_3D = 128
STEP_SOURCES = ("rt_step3.hpp", "rt_common.hpp", "rt_internal.hpp", "rt_kernels.inc",
                "rt_kernels_f64.hip", "rt_kernels_f32.hip", "rt_step3_inst.inc") + tuple(
                    f"rt_step3_{p}_g{g}.hip" for p in ("f64", "f32") for g in (1, 2, 3, 4))


def algorithmic_bytes_per_cell(nang: int, sbytes: int) -> int:
    """I read once and written once per angle, plus the per-cell fields."""
    return 2 * sbytes * nang + FIELD_BYTES_PER_CELL


def _code_only(text: str) -> str:
    """C++ source without its comments, blank lines and indentation (string
    literals in these files hold no comment markers)."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.strip() for line in text.splitlines() if line.strip())


def kernel_source_sha() -> str:
    """Digest of the fused step kernel's code (comments aside) and build
    flags: counters taken on another kernel do not describe this one."""
    import hashlib

    from paper_1403_6126_amd import build as B
    h = hashlib.sha256()
    for name in STEP_SOURCES:
        with open(os.path.join(B.CSRC, name), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    h.update(" ".join(B.HIPCC_FLAGS).encode())
    h.update(json.dumps(B.EXTRA_FLAGS, sort_keys=True).encode())
    return h.hexdigest()[:16]


def load_traffic(tag: str, workload: str):
    """HBM bytes per launch of the fused kernel from rocprofv3 FETCH_SIZE and
    WRITE_SIZE counters, as committed under profiles/ (file name returned as
    the source), or None when no summary exists or it was taken on other
    kernel sources than the ones built now."""
    rel = os.path.join("profiles", f"traffic_{tag}_{workload}.json")
    path = os.path.join(ROOT, rel)
    if not os.path.exists(path):
        return None, None
    try:
        with open(path) as f:
            d = json.load(f)
    except Exception:
        return None, None
    if d.get("kernel_source_sha") != kernel_source_sha():
        return None, rel + " (taken on other kernel sources)"
    return d.get("bytes_per_launch"), rel


def kernel_name(info, storage_bytes: int) -> str:
    """The fused kernel instance of a context's launch shape."""
    t = "double" if storage_bytes == 8 else "float"
    waves = max(1, info["block_threads"] // 64)
    ng = -(-info["nang"] // 10)
    groups = -(-ng // waves)
    per = "true" if info.get("periodic", True) else "false"
    so = "true" if info.get("second_order", False) else "false"
    return f"rtk::k_step3<{t}, {t}, 10, {groups}, {per}, true, {so}>"


def rooflines(r, tag: str, wname: str):
    """HBM roofline (algorithmic bytes over the kernel time against the 8 TB/s
    peak, with the counters' traffic) and VALU-issue roofline (algorithmic
    operations over the kernel time against the issue peak) of one run."""
    traffic, source = load_traffic(tag, wname)
    kname = kernel_name(r, r["storage_bytes"])
    upd_per_s = r["updates_per_launch"] / (r["kernel_ms"] * 1e-3)
    ops = ALG_OPS_PER_CELL_ANGLE_3D * upd_per_s
    hbm = {"bound": "hbm", "achieved": r["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": r["achieved_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
           "traffic_source": source, "kernel": kname, "kernel_ms": r["kernel_ms"],
           "bytes_per_launch": r["bytes_per_launch"]}
    alu = {"bound": "alu", "achieved": ops / 1e12, "peak": VALU_ISSUE_PEAK / 1e12,
           "unit": "Tops/s (VALU issue)", "frac": ops / VALU_ISSUE_PEAK,
           "ops_per_cell_angle": ALG_OPS_PER_CELL_ANGLE_3D, "kernel": kname}
    return hbm, alu


def run_gpu(wl, precision: str, steps: int, warmup: int, second_order: bool = False):
    import torch

    import workloads as W
    from paper_1403_6126_amd import rt
    from paper_1403_6126_amd.solver import Solver, quadrature_for

    mu, w = quadrature_for(wl.quad)
    if "E0" in wl.meta:   # I = (E + 3 n.F)/(4 pi), built on the device
        E = torch.as_tensor(wl.meta["E0"], device="cuda")
        F = torch.as_tensor(wl.meta["F0"], device="cuda")
        I0 = W.moment_intensity(torch.as_tensor(mu, device="cuda"), E, F, xp=torch)
        del E, F
    else:                 # I = T^4/(4 pi), an expanded view
        T = torch.as_tensor(wl.T).cuda()
        I0 = W.equilibrium_intensity(T, len(w), xp=torch)
    s = Solver(wl, precision=precision, mu=mu, w=w, I0=I0, second_order=second_order)
    del I0
    torch.cuda.empty_cache()
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
                grid_blocks=info.grid_blocks, block_threads=info.block_threads,
                updates_per_launch=wl.ncell * info.nang,
                periodic=all(b[0] == 0 for b in wl.bc[:wl.ndim]))


def _host_cpu():
    """Thread count and processor model of the host the oracle runs on."""
    model = ""
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    return os.cpu_count(), model


def cpu_baseline(threads: int = 0):
    """The CPU oracle (as it stands, plain FP64 C) timed on the host: steps
    only, the workload already in memory.  One full step of the 128^3 S8 box
    (the GPU line's workload) on all threads, and the 512-cell GL16 slab
    (100 steps) on one thread and on all threads."""
    import oracle
    import workloads as W

    nproc, model = _host_cpu()
    if threads > 0:
        oracle.set_threads(threads)
    nthr = oracle.threads()

    def rate(wl, nsteps):
        st = oracle.State(oracle.Problem(wl))
        t0 = time.perf_counter()
        st.step(nsteps=nsteps)
        el = time.perf_counter() - t0
        return wl.ncell * st.prob.nang * nsteps / el, el

    slab = W.config1()
    oracle.set_threads(1)
    r1, t1 = rate(slab, 100)
    oracle.set_threads(nthr)
    rn, tn = rate(slab, 100)
    box = W.config2()
    rb, tb = rate(box, 1)
    return dict(value=rb, unit="cell-angle updates/s", cores=nthr, kind="oracle",
                sample=f"one full step of the 128^3 S8 FP64 box on {nthr} threads, steps only "
                       f"({tb:.1f} s)",
                per_core=rb / nthr, nproc=nproc, cpu_model=model,
                slab_512_gl16_100_steps={"threads_1": r1, f"threads_{nthr}": rn,
                                         "seconds": [t1, tn]})


def configs_leg(steps: int = 5, warmup: int = 2):
    """The FP32-mixed fused step on the other full-size workloads: the 256^3
    shadow box (fixed faces, beam, clump) and the 512x512x256 advective
    diffusion box.  Kernel time from the same HIP events as the main line."""
    import torch

    import workloads as W
    out = {}
    for name, make in (("shadow3d_256cube_S8_fixed", lambda: W.config3(nper=256)),
                       ("diffusion3d_512x512x256_S8", lambda: W.config5())):
        print(f"bench: {name} mixed warmup={warmup} steps={steps}", file=sys.stderr, flush=True)
        wl = make()
        r = run_gpu(wl, "mixed", steps, warmup)
        del wl
        torch.cuda.empty_cache()
        hbm, alu = rooflines(r, "k_step3_mixed", name)
        out[name] = dict(value=r["value"], ms_per_step=r["ms_per_step"], kernel_ms=r["kernel_ms"],
                         cells=r["updates_per_launch"] // r["nang"], angles=r["nang"],
                         roofline=hbm, compute_roofline=alu)
        print(f"bench: {name} {r['value']:.4g} cell-angle/s, kernel {r['kernel_ms']:.3f} ms",
              file=sys.stderr, flush=True)
    return out


# A packed solve runs on one workgroup: beyond about 512 cells its single CU,
# not the device, sets its latency (packed requests of up to 4096 cells had a
# median latency of 0.5 s on the 200-request trace at load 0.8, against 20 ms
# at 512).
SERVE_DEFAULTS = dict(pool_bytes=96 << 30, max_active=1024, packed_cells=512,
                      chunk_work=400_000_000, large_work=40_000_000)


def serving(count: int, loads, warm: int, seed: int = 4, fifo: bool = True):
    """The serving stream: `count` requests of the mixed-size trace (1D/2D/3D
    grids of 64 to 128^3 cells log-uniform, 16-288 directions, 10-200 steps,
    FP32-mixed, Poisson arrivals).  The batched capacity is measured first in
    a closed loop over the first `warm` requests; for each offered load (times
    that capacity) the arrivals are scaled to it and the same trace runs
    through the server and through the plain one-at-a-time path.  The
    capacity run takes the whole trace by default: a prefix of a heavy-tailed
    mix need not carry its mean cost.  Latencies are also given per request
    class (packed, chunked, large)."""
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
    runs = {}
    for load in loads:
        rate = load * cap["throughput"] / work.mean()          # requests per second
        arrivals = np.cumsum([r["gap"] for r in reqs]) / rate
        arrivals -= arrivals[0]
        print(f"bench: serving capacity {cap['throughput']:.3g} updates/s, load {load}: offered "
              f"{rate:.3g} req/s over {arrivals[-1]:.1f} s", file=sys.stderr, flush=True)
        b = serve.run_batched(wls, arrivals, progress=say, **SERVE_DEFAULTS)
        print(f"bench: served p50 {b['latency_p50_s']*1e3:.1f} ms p99 "
              f"{b['latency_p99_s']*1e3:.1f} ms {b['throughput']:.3g} updates/s", file=sys.stderr,
              flush=True)
        torch.cuda.empty_cache()
        f = None
        if fifo:
            f = serve.run_fifo(wls, arrivals, progress=say,
                               packed_cells=SERVE_DEFAULTS["packed_cells"],
                               large_work=SERVE_DEFAULTS["large_work"])
            print(f"bench: fifo p50 {f['latency_p50_s']*1e3:.1f} ms p99 "
                  f"{f['latency_p99_s']*1e3:.1f} ms {f['throughput']:.3g} updates/s",
                  file=sys.stderr, flush=True)
        runs[f"load_{load}"] = dict(load=load, offered_req_per_s=rate, batched=b, fifo=f)
    return dict(requests=count, closed_loop_capacity=cap["throughput"],
                mean_updates_per_request=float(work.mean()), runs=runs, server=SERVE_DEFAULTS,
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
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the FP32-mixed timing of the 256^3 shadow and 512x512x256 "
                         "diffusion boxes")
    ap.add_argument("--only-configs", action="store_true",
                    help="profiling: run the shadow and diffusion timing alone")
    ap.add_argument("--config-steps", type=int, default=5,
                    help="timed steps of the shadow and diffusion boxes")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the CPU-baseline leg (0: all host threads)")
    ap.add_argument("--only-cpu", action="store_true",
                    help="run the CPU-baseline leg alone (no GPU) and print its JSON")
    ap.add_argument("--only", choices=["fp64", "mixed"], default=None,
                    help="profiling: run one precision only and print its timing")
    ap.add_argument("--second-order", action="store_true",
                    help="with --only: time the step with the absorption system solved twice "
                         "(second-order absorption)")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="requests of the serving trace (0: skip; 2000 = the full stream)")
    ap.add_argument("--serve-load", type=float, nargs="+", default=[0.8, 1.2],
                    help="offered loads relative to the closed-loop capacity (the trace is "
                         "replayed at each)")
    ap.add_argument("--serve-warm", type=int, default=0,
                    help="requests of the closed-loop capacity run (0: the whole trace)")
    ap.add_argument("--only-serve", action="store_true")
    ap.add_argument("--serve-packed-cells", type=int, default=SERVE_DEFAULTS["packed_cells"],
                    help="largest FP32 request (cells) run in packed persistent launches")
    ap.add_argument("--serve-large-work", type=int, default=SERVE_DEFAULTS["large_work"],
                    help="updates per step from which a request takes the large stream")
    ap.add_argument("--serve-chunk-work", type=int, default=SERVE_DEFAULTS["chunk_work"],
                    help="cell-angle updates per chunked launch group")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="profiling: time a plain device-to-device copy of this many GiB "
                         "(counter calibration) and exit")
    args = ap.parse_args()
    SERVE_DEFAULTS.update(packed_cells=args.serve_packed_cells, large_work=args.serve_large_work,
                          chunk_work=args.serve_chunk_work)
    if args.second_order and not args.only:
        ap.error("--second-order goes with --only")
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the library "
              "has no multi-GPU path (the domain decomposition it would use is a design, "
              "not code)", file=sys.stderr)
        sys.exit(2)
    if args.only_cpu:
        print(json.dumps(cpu_baseline(threads=args.cpu_threads)), flush=True)
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
    if args.only_configs:
        print(json.dumps(configs_leg(steps=args.config_steps)), flush=True)
        return
    if args.only_serve:
        print(json.dumps(serving(args.serve_requests, args.serve_load, args.serve_warm)),
              flush=True)
        return
    wl = W.config2(nper=args.nper)
    wname = f"box3d_{args.nper}cube_S8"
    print(f"bench: {wname} {args.only or 'fp64'} warmup={args.warmup} steps={args.steps}",
          file=sys.stderr, flush=True)
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
        hbm, alu = rooflines(rmx, "k_step3_mixed", wname)
        mixed = dict(value=rmx["value"], ms_per_step=rmx["ms_per_step"], dtype="f32 (I), f64 (T)",
                     roofline=hbm, compute_roofline=alu)
    others = None
    if not args.no_configs:
        torch.cuda.empty_cache()
        others = configs_leg(steps=args.config_steps)
    srv = None
    if args.serve_requests > 0:
        torch.cuda.empty_cache()
        srv = serving(args.serve_requests, args.serve_load, args.serve_warm)
    cpu = None
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(threads=args.cpu_threads)
    hbm64, alu64 = rooflines(r64, "k_step3_fp64", wname)
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
        "roofline": hbm64,
        "compute_roofline": alu64,
        "fp32_mixed": mixed,
        "fp32_mixed_other_workloads": others,
        "serving": srv,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
