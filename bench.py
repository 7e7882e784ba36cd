"""Benchmark: twisted Wilson flow throughput on one MI355X.

One step = one pass of the whole hot path over one batch: ingest of the
canonical FP64 links of every configuration (pack into device storage +
SU(3) check) followed by the full flow of the batch to its t_end with RK3
steps of eps = 0.01, FP64 measurements of t^2 E, plaquette and Q every 0.1
and at t_end, all stage launches of the batch captured in one HIP graph.

Default workload (ensemble batch): 64 configurations of 8x8x24x24, 16 of
6x6x18x18 and 16 of 10x10x30x30, twist n_01 = 1, seeded near-identity links
exp(i eps H) with eps in {0.2, 0.3, 0.4}, flowed to c = 0.3 (t_end =
c^2 L^2 / 8), FP32 storage with 12-real links, FP64 reunitarisation every
10 steps.  The same batch is also flowed with the plain FP64 path.
`--workload large` runs one 32x32x96x96 box (t_end 11.52, measured every 0.1;
with --large-steps N only its first N steps).

Prints one JSON line (metric, value = site-updates/s, roofline, cpu_baseline).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "flowed site-updates/s + HBM GB/s (FP32 batched vs FP64 plain) at t^2E err<=1e-5"
EPS = 0.01
HBM_PEAK_GBS = 8000.0
# Published MI355X vector peaks (TFLOP/s): FP32 157.3 (with packed FP32), FP64 78.6.
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6
# Non-packed FMA issue: 256 CU x 64 lanes x 2 flop x 2.4 GHz.  The build turns
# packed FP32 off, so this is what the FP32 kernels can issue at most.
ALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
LARGE_STEPS = 100


def host_cpu():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def batch_workload():
    """(dims, link-eps, seed, t_end) per configuration."""
    cfgs = []
    j = 0
    for L, count in ((8, 64), (6, 16), (10, 16)):
        for _ in range(count):
            cfgs.append(((L, L, 3 * L, 3 * L), (0.2, 0.3, 0.4)[j % 3], 4000 + j,
                         0.09 * L * L / 8))
            j += 1
    return cfgs


def large_workload(steps=None):
    """One 32x32x96x96 Haar box flowed to c = 0.3 (t_end 11.52), or only the
    first `steps` steps of that flow."""
    t_end = 0.09 * 32 * 32 / 8 if steps is None else steps * EPS
    return [((32, 32, 96, 96), None, 5, t_end)]


def n_steps(t_end, t0=0.0):
    n = 0
    while t0 + (n + 1) * EPS <= t_end + 1e-12:
        n += 1
    return n + (1 if t_end - (t0 + n * EPS) > 1e-12 else 0)


# Algorithmic work per site per RK3 step (3 stages): every link and accumulator
# element an RK stage touches, once, with ping-pong link buffers.
def bytes_per_site_step(storage, variant="site"):
    ne, cb = (6, 8) if storage == "f32c12" else ((9, 8) if storage == "f32" else (9, 16))
    links = 3 * 2 * 4 * ne * cb           # read + write every stage
    x = (1 + 2 + 1) * 4 * 4 * cb          # X: write, read+write, read
    return links + x


MM = 198.0            # 3x3 complex product: 27 complex multiplies + 18 complex adds
R2 = 132.0            # rows 0,1 of a 3x3 complex product
REBUILD = 42.0        # row 2 = conj(row0 x row1): 6 complex multiplies + 3 subtractions
EXP, XUPD = 300.0, 56.0


def flops_per_site_stage(storage, variant):
    """Real FP operations per site for one RK stage, by kernel."""
    c12 = storage == "f32c12"
    upd = R2 if c12 else MM
    if variant.startswith(("site_alg", "site_lds", "site_plq")):
        if storage == "f64":
            # six two-row plaquettes projected to su(3) (r2_proj_ah ~55, +-accumulate 16),
            # twelve lower staples (a product and an accumulated product, 2 MM + 18),
            # four U S products + projection (16)
            return (18 * R2 + 6 * (55 + 16) + 12 * (2 * MM + 18) + 4 * (MM + 16)
                    + 4 * (EXP + upd + XUPD))
        # FP32: six upper plaquettes and twelve lower closed loops, three two-row
        # products each, projected (55) and accumulated (16 for the two links of an
        # upper plaquette, 8 for a lower loop); 12-real storage rebuilds the third
        # row of every non-leading factor (15 in the upper plaquettes, where each
        # own link is rebuilt once, and 36 in the lower loops)
        return (54 * R2 + 6 * (55 + 16) + 12 * (55 + 8) + 4 * (EXP + upd + XUPD)
                + (REBUILD * 51 if c12 else 0))
    if variant.startswith("site"):
        return 46 * MM + 4 * (EXP + upd + XUPD) + (REBUILD * 44 if c12 else 0)
    # one thread per link: six staples and U S per link
    return 4 * (13 * MM + EXP + upd + XUPD) + (REBUILD * 4 * 19 if c12 else 0)


def flops_per_site_step(storage, variant):
    return 3 * flops_per_site_stage(storage, variant)


def kernel_source_hash(root=ROOT):
    """Hash of the stage kernels' code (comments and blank lines left out, so
    that a profile stays valid across comment edits but not across a change
    of the code)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("kernels.hip", "lattice_dev.h", "su3_dev.h", "layout.h"):
        with open(os.path.join(root, "paper_2107_03747_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        lines = [ln.rstrip() for ln in text.splitlines() if ln.strip()]
        h.update("\n".join(lines).encode())
    return h.hexdigest()[:16]


def profiled_traffic(variant, storage, workload):
    """Counter-based HBM bytes per stage launch from profiles/*_hbm.md, when
    that summary was taken on the current kernel sources, variant and workload."""
    import glob
    want = kernel_source_hash()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_hbm.md"))):
        meta = {}
        with open(path) as fh:
            for line in fh:
                if ":" in line and not line.startswith(("|", "#", " ", "`")):
                    k, v = line.split(":", 1)
                    meta[k.strip()] = v.strip()
        if (meta.get("kernel-source-sha256-16") == want and meta.get("variant") == variant
                and meta.get("storage", "f32c12") == storage
                and meta.get("workload", "batch") == workload
                and "traffic_bytes_per_launch" in meta):
            return float(meta["traffic_bytes_per_launch"]), os.path.basename(path)
    return None, None


def make_inputs(cfgs, device):
    from paper_2107_03747_amd import gen
    out = []
    for dims, e, seed, _ in cfgs:
        if e is None:
            out.append(gen.haar(dims, seed, device=device))
        else:
            out.append(gen.near_identity(dims, e, seed, device=device))
    return out


def time_flows(tgf, torch, cfgs, inputs, storage, steps, warmup, flags=0, reunit=10,
               variant=None):
    t_end = [c[3] for c in cfgs]
    f = tgf.Flow([c[0] for c in cfgs], storage)
    f.load_all(inputs)
    if variant is None:
        f.autotune(None)
    else:
        f.set_variant(variant)

    def one():
        f.load_all(inputs)
        return f.flow(EPS, t_end, 0.1, reunit, flags)

    rows = None
    for _ in range(warmup):
        rows = one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        rows = one()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(steps, 1)
    return f, rows, dt


def cpu_baseline(cfgs, inputs, gpu_rows, target_s=12.0, single_s=6.0):
    """The FP64 oracle on a bounded sample of the same workload: whole flows of
    the first configurations of the batch (each from t = 0 to its t_end with
    rows only at t_end) on all host threads, as many as fit in about
    target_s, and the first steps of configuration 0 on one thread (about
    single_s); the sample's t^2 E at t_end is also compared with the GPU rows
    of the timed run."""
    import numpy as np

    import oracle
    oracle.build(force=False)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # one thread: steps of config 0 until about single_s
    dims0 = cfgs[0][0]
    V0 = int(np.prod(dims0))
    oracle.set_threads(1)
    U = inputs[0].cpu().numpy().copy()
    t = time.perf_counter()
    oracle.rk3_step(U, dims0, EPS)
    n1 = max(1, int(single_s / (time.perf_counter() - t)))
    U = inputs[0].cpu().numpy().copy()
    t = time.perf_counter()
    oracle.flow(U, dims0, EPS, n1 * EPS, 0.0)
    dt1 = time.perf_counter() - t
    single = {"value": V0 * n1 / dt1, "unit": "site-updates/s", "cores": 1,
              "sample": f"config 0 ({'x'.join(map(str, dims0))}), first {n1} FP64 RK3 steps: "
                        f"{V0 * n1} site-updates in {dt1:.1f} s"}
    oracle.set_threads(threads)
    done, su, elapsed, errs = 0, 0, 0.0, []
    while done < len(cfgs) and (done == 0 or elapsed * (done + 1) / done <= target_s):
        dims, _, _, t_end = cfgs[done]
        U = inputs[done].cpu().numpy().copy()
        t = time.perf_counter()
        rows = oracle.flow(U, dims, EPS, t_end, 0.0)
        elapsed += time.perf_counter() - t
        su += int(np.prod(dims)) * n_steps(t_end)
        last = [r for r in range(gpu_rows.shape[0]) if abs(gpu_rows[r, done, 0] - rows[-1, 0]) < 1e-9]
        if last:
            g = gpu_rows[last[0], done, 2]
            errs.append(abs(g - rows[-1, 2]) / abs(rows[-1, 2]))
        done += 1
    shapes = sorted({"x".join(map(str, c[0])) for c in cfgs[:done]})
    return {
        "value": su / elapsed,
        "unit": "site-updates/s",
        "cores": oracle.get_threads(), "host_cpu": host_cpu(), "host_nproc": os.cpu_count(),
        "kind": "oracle",
        "sample": f"configs 0..{done - 1} of the batch ({', '.join(shapes)}), whole FP64 flows "
                  f"with eps={EPS} from t=0 to t_end and one measurement each: {su} site-updates "
                  f"in {elapsed:.1f} s",
        "single_thread": single,
    }, (max(errs) if errs else None), done


# Monte Carlo (hybrid over-relaxation, FP64 full storage), per link update.
# Bytes: one launch updates the V/2 links of one direction and parity and
# needs every link of the lattice once (the three other directions at all
# sites, its own direction at both parities) and writes V/2 links:
# (4 V + V/2) x 144 B / (V/2) = 1296 B.  Flops: six staples (2484), Omega
# (198), three subgroup updates (3 x 240); the heat bath's random numbers and
# acceptance tests (integer Philox, log, cos) are not counted.
MC_BYTES_PER_LINK = (4 + 0.5) * 144 / 0.5
MC_FLOPS_PER_LINK = 2484 + 198 + 3 * 240
MC_B = 0.5
MC_N_OR = 3
MC_CPU_CFGS = 64


def time_mc(tgf, torch, cfgs, inputs, reps, cpu=True):
    """Hybrid sweeps (1 heat bath + MC_N_OR over-relaxation) on the batch
    geometry in FP64: wall time of `reps` hybrid sweeps after one warm-up.
    cpu: also run the oracle's Monte Carlo on the first MC_CPU_CFGS
    configurations for the warm-up hybrid sweep (same seed and counters) --
    its time is the CPU baseline and its links are compared with the GPU's."""
    f = tgf.Flow([c[0] for c in cfgs], "f64")
    f.load_all(inputs)
    sw = f.mc(MC_B, 1, MC_N_OR, seed=1)
    torch.cuda.synchronize()
    first = [f.store(k).cpu().numpy() for k in range(MC_CPU_CFGS)] if cpu else None
    t0 = time.perf_counter()
    for _ in range(reps):
        sw = f.mc(MC_B, 1, MC_N_OR, seed=1, sweep0=sw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sweeps = reps * (1 + MC_N_OR)
    links = 4 * sum(math.prod(c[0]) for c in cfgs)
    rate = links * sweeps / dt
    launch_ms = dt / (8 * sweeps) * 1e3
    gbs = rate * MC_BYTES_PER_LINK / 1e9
    tflops = rate * MC_FLOPS_PER_LINK / 1e12
    out = {
        "metric": "Monte Carlo link-updates/s (hybrid over-relaxation, FP64)",
        "value": round(rate, 1),
        "unit": "link-updates/s",
        "b": MC_B,
        "sweeps": sweeps,
        "heatbath_per_hybrid": 1,
        "overrelax_per_hybrid": MC_N_OR,
        "ms_per_sweep": round(dt / sweeps * 1e3, 3),
        "roofline": {
            "kernel": "mc_kernel<mu>",
            "bound": "hbm",
            "achieved": round(gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4),
            "alu_tflops": round(tflops, 2),
            "alu_frac_fp64": round(tflops / ALU_PEAK_TFLOPS, 4),
            "avg_launch_ms_wall": round(launch_ms, 4),
            "bytes_per_link_update": MC_BYTES_PER_LINK,
            "flops_per_link_update": MC_FLOPS_PER_LINK,
        },
    }
    if cpu:
        import numpy as np
        import oracle
        oracle.build(force=False)
        oracle.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
        tc, n, dmax = 0.0, 0, 0.0
        for k in range(MC_CPU_CFGS):
            d = cfgs[k][0]
            U = inputs[k].cpu().numpy().copy()
            t0 = time.perf_counter()
            oracle.mc(U, d, MC_B, 1, MC_N_OR, 1, sweep0=0, cfg=k)
            tc += time.perf_counter() - t0
            n += 4 * math.prod(d) * (1 + MC_N_OR)
            dmax = max(dmax, float(np.abs(first[k] - U).max()))
        out["cpu_baseline"] = {"value": round(n / tc, 1), "unit": "link-updates/s",
                               "cores": oracle.get_threads(), "host_cpu": host_cpu(), "kind": "oracle",
                               "sample": f"configurations 0..{MC_CPU_CFGS - 1} of the batch "
                                         f"(8x8x24x24), one hybrid sweep each (1 HB + "
                                         f"{MC_N_OR} OR): {n} link updates in {tc:.2f} s"}
        out["max_abs_dU_vs_oracle_sample"] = dmax
    return out


# General SU(N) (FP64, row-per-lane kernels), per site per RK3 step.
# Bytes: links read + written every stage, 3 x 2 x 4 x N^2 x 16, and the full
# N x N accumulator X written, read + written, read: 4 x 4 x N^2 x 16.
# Flops: per link and stage 25 N x N products (6 staples of 2, U S, 11 Horner
# steps of the exponential, exp(X) U) of 8 N^3 flop, plus the staple sums
# (6 N^2 complex multiply-adds), P_ah and the RK update (~2 N^2 of them).
def sun_bytes_per_site_step(N):
    return 3 * 2 * 4 * N * N * 16 + 4 * 4 * N * N * 16


def sun_flops_per_site_step(N):
    return 4 * 3 * (25 * 8 * N ** 3 + 8 * 8 * N * N)


def sun_mode(tgf, torch, args):
    """SU(N) flow of a batch of l^2 x (N l)^2 boxes (the TGF geometry), l =
    args.sun_l, twist k = 1, near-identity links, about args.sun_sites sites in
    total, flowed for args.sun_steps steps of eps; site-updates/s, the stage
    kernel's HIP-event average and its ALU roofline."""
    from paper_2107_03747_amd import gen
    N, l = args.nc, args.sun_l
    d = (l, l, N * l, N * l)
    V = math.prod(d)
    n_cfg = max(1, args.sun_sites // V)
    log(f"SU({N}): {n_cfg} x {'x'.join(map(str, d))}")
    links = [gen.near_identity_n(d, N, 0.3, seed=6000 + k, device="cuda") for k in range(n_cfg)]
    t_end = args.sun_steps * EPS
    f = tgf.Flow([d] * n_cfg, "f64", nc=N)
    f.load_all(links)
    v = f.autotune(None) if args.variant is None else args.variant
    f.set_variant(v)
    rows_per_lane = int(tgf.tgf_sun_rows_per_lane(N, v))
    lds = int(tgf.tgf_sun_variant_lds(N, v)) == 1
    log(f"SU({N}): variant {v} ({rows_per_lane} rows per lane, "
        f"{'LDS operands' if lds else 'permutes'})")
    f.flow(EPS, t_end, 0.0)                      # warm-up (graph capture)
    times = []
    for _ in range(max(1, args.steps // 5)):
        f.load_all(links)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rows = f.flow(EPS, t_end, 0.0)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    dt = min(times)
    site_updates = n_cfg * V * args.sun_steps
    f.load_all(links)
    f.flow(EPS, t_end, 0.0, 0, tgf.TGF_TIMING)
    tm = f.timing()
    stage_ms = tm["stage_ms"] / tm["stage_launches"]
    site_stages = 3 * tm["stage_site_updates"] / tm["stage_launches"]
    tflops = site_stages * sun_flops_per_site_step(N) / 3 / (stage_ms * 1e-3) / 1e12
    gbs = site_stages * sun_bytes_per_site_step(N) / 3 / (stage_ms * 1e-3) / 1e9
    out = {
        "metric": f"SU({N}) flowed site-updates/s (FP64)",
        "value": round(site_updates / dt, 1),
        "unit": "site-updates/s",
        "nc": N,
        "ms_per_flow": round(dt * 1e3, 3),
        "config": {"workload": f"{n_cfg} x {'x'.join(map(str, d))}, twist k=1, near-identity "
                               f"links eps 0.3, {args.sun_steps} steps of {EPS}",
                   "n_configs": n_cfg, "sites": n_cfg * V},
        "t2E_last_cfg0": float(rows[-1, 0, 2]),
        "rows_per_lane": rows_per_lane,
        "operands": "lds" if lds else "permutes",
        "roofline": {"kernel": (f"sun_stage_lds_kernel<{N}>" if lds
                                else f"sun_stage_kernel<{N}, {rows_per_lane}>"), "bound": "alu",
                     "achieved": round(tflops, 3), "peak": round(ALU_PEAK_TFLOPS, 1),
                     "unit": "TFLOP/s", "frac": round(tflops / ALU_PEAK_TFLOPS, 4),
                     "hbm_gbs_algorithmic": round(gbs, 1),
                     "avg_launch_ms": round(stage_ms, 4),
                     "flops_per_site_step": sun_flops_per_site_step(N),
                     "bytes_per_site_step": sun_bytes_per_site_step(N)},
    }
    if not args.no_cpu:
        import numpy as np
        import oracle
        oracle.build(force=False)
        oracle.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
        U = links[0].cpu().numpy().copy()
        k = max(1, min(args.sun_steps, 3))
        t0 = time.perf_counter()
        ref = oracle.sun_flow(U, d, EPS, k * EPS, 0.0)
        tc = time.perf_counter() - t0
        g = tgf.Flow([d], "f64", nc=N)
        g.set_variant(v)
        g.load(0, links[0])
        rg = g.flow(EPS, k * EPS, 0.0)
        out["cpu_baseline"] = {"value": round(V * k / tc, 1), "unit": "site-updates/s",
                               "cores": oracle.get_threads(), "host_cpu": host_cpu(),
                               "kind": "oracle",
                               "sample": f"configuration 0, {k} steps: {V * k} site-updates "
                                         f"in {tc:.2f} s"}
        out["t2E_gpu_oracle_sample"] = [float(rg[-1, 0, 2]), float(ref[-1, 2])]
        out["t2E_rel_err_vs_oracle_sample"] = float(abs(rg[-1, 0, 2] - ref[-1, 2]) /
                                                    abs(ref[-1, 2]))
    print(json.dumps(out), flush=True)


def copy_mode(tgf, torch, args):
    """Plain copy of a known size with the library's copy kernel: reads and
    writes `bytes` each per launch.  Used to calibrate the HBM counters."""
    nbytes = int(args.copy_gib * (1 << 30)) // 16 * 16
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.random_(0, 255)
    dst = torch.empty_like(src)
    for _ in range(args.warmup):
        tgf.stream_copy(dst, src, nbytes)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        tgf.stream_copy(dst, src, nbytes)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    print(json.dumps({"mode": "copy", "bytes_per_launch_read": nbytes,
                      "bytes_per_launch_written": nbytes, "launches": args.steps,
                      "ms_per_launch": round(dt * 1e3, 4),
                      "copy_gbs": round(2 * nbytes / dt / 1e9, 1)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=("batch", "large"), default="batch")
    ap.add_argument("--storage", choices=("f32c12", "f32", "f64"), default="f32c12")
    ap.add_argument("--variant", type=int, default=None)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-mc", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--large-steps", type=int, default=None,
                    help=f"steps of the 32x32x96x96 leg (default {LARGE_STEPS}); with "
                         "--workload large, flow only this many steps (default: the whole flow)")
    ap.add_argument("--mc-reps", type=int, default=3)
    ap.add_argument("--mode", choices=("flow", "copy", "mc", "sun"), default="flow",
                    help="copy: time the library's plain HBM copy kernel (counter calibration); "
                         "mc: time only the Monte Carlo on the batch geometry; "
                         "sun: time the general SU(N) flow (--nc)")
    ap.add_argument("--nc", type=int, default=4)
    ap.add_argument("--sun-l", type=int, default=4)
    ap.add_argument("--sun-sites", type=int, default=1 << 20)
    ap.add_argument("--sun-steps", type=int, default=20)
    ap.add_argument("--copy-gib", type=float, default=2.0)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2107_03747_amd import tgf

    if args.mode == "copy":
        copy_mode(tgf, torch, args)
        return
    if args.mode == "sun":
        sun_mode(tgf, torch, args)
        return

    cfgs = batch_workload() if args.workload == "batch" else large_workload(args.large_steps)
    args.no_large = args.no_large or args.workload != "batch"
    log(f"generating {len(cfgs)} configurations on the GPU")
    inputs = make_inputs(cfgs, "cuda")
    torch.cuda.synchronize()
    if args.mode == "mc":
        log(f"timing the Monte Carlo: {args.mc_reps} hybrid sweeps")
        print(json.dumps(time_mc(tgf, torch, cfgs, inputs, args.mc_reps, cpu=not args.no_cpu)),
              flush=True)
        return
    site_updates = sum(math.prod(c[0]) * n_steps(c[3]) for c in cfgs)
    sites = sum(math.prod(c[0]) for c in cfgs)

    log(f"timing {args.storage}: {args.warmup} warmup + {args.steps} steps")
    f, rows, dt = time_flows(tgf, torch, cfgs, inputs, args.storage, args.steps, args.warmup,
                             variant=args.variant)
    variant = tgf.variant_names()[f.variant]
    value = site_updates / dt
    log("kernel timing pass")
    roofline = stage_roofline(tgf, f, cfgs, inputs, args.storage, variant, args.workload)
    whole_gbs = site_updates * bytes_per_site_step(args.storage, variant) / dt / 1e9

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.storage == "f64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": ("ensemble batch: 64 x 8x8x24x24 + 16 x 6x6x18x18 + 16 x 10x10x30x30, "
                         "twist n01=1, near-identity links eps {0.2,0.3,0.4}, flow to c=0.3")
                        if args.workload == "batch" else
                        ("large box 32x32x96x96, twist n01=1, Haar links, " +
                         ("flow to c=0.3" if args.large_steps is None else
                          f"first {args.large_steps} RK3 steps of the flow to c=0.3")),
            "n_configs": len(cfgs),
            "sites": sites,
            "site_updates_per_step": site_updates,
            "storage": args.storage,
            "eps": EPS,
            "meas_dt": 0.1,
            "reunit_every": 10,
            "variant": variant,
            "lds_block_sites": block_shapes(f, cfgs),
            "hip_graph": True,
        },
        "roofline": roofline,
        "hbm_gbs_whole_pass": round(whole_gbs, 1),
        "hbm_frac_whole_pass": round(whole_gbs / HBM_PEAK_GBS, 4),
    }

    if not args.no_fp64 and args.storage == "f32c12":
        log("timing the FP32 full-matrix storage on the same workload")
        del f
        torch.cuda.empty_cache()
        k32 = max(1, args.steps // 3)
        f32, rows32, dt32 = time_flows(tgf, torch, cfgs, inputs, "f32", k32, 1)
        v32 = tgf.variant_names()[f32.variant]
        out["fp32_full"] = {"value": round(site_updates / dt32, 1), "unit": "site-updates/s",
                            "ms_per_step": round(dt32 * 1e3, 3), "steps": k32, "variant": v32,
                            "bytes_per_site_step": bytes_per_site_step("f32", v32),
                            "lds_block_sites": block_shapes(f32, cfgs)}
        f = f32            # freed with the FP64 leg below
    else:
        rows32, dt32 = None, None

    if not args.no_fp64 and args.storage != "f64":
        log("timing FP64 plain path on the same workload")
        del f
        torch.cuda.empty_cache()
        k64 = max(1, args.steps // 3)
        f64, rows64, dt64 = time_flows(tgf, torch, cfgs, inputs, "f64", k64, 1)
        pos = rows64[:, :, 0] > 0
        rel = np.abs(rows[:, :, 2] - rows64[:, :, 2])[pos] / np.abs(rows64[:, :, 2][pos])
        out["fp64_plain"] = {"value": round(site_updates / dt64, 1), "unit": "site-updates/s",
                             "ms_per_step": round(dt64 * 1e3, 3), "steps": k64,
                             "variant": tgf.variant_names()[f64.variant],
                             "lds_block_sites": block_shapes(f64, cfgs)}
        out["speedup_vs_fp64_plain"] = round(dt64 / dt, 3)
        out["t2E_max_rel_err_vs_fp64_gpu"] = float(rel.max())
        if rows32 is not None:
            rel32 = np.abs(rows32[:, :, 2] - rows64[:, :, 2])[pos] / np.abs(rows64[:, :, 2][pos])
            out["fp32_full"]["speedup_vs_fp64_plain"] = round(dt64 / dt32, 3)
            out["fp32_full"]["t2E_max_rel_err_vs_fp64_gpu"] = float(rel32.max())
        del f64
        torch.cuda.empty_cache()

    if args.workload == "batch" and not args.no_large:
        large_steps = args.large_steps or LARGE_STEPS
        log(f"large box: first {large_steps} steps of 32x32x96x96, FP32 12-real and FP64")
        out["large"] = large_leg(tgf, torch, np, large_steps)

    if not args.no_mc:
        log("timing the Monte Carlo on the same geometry")
        out["mc"] = time_mc(tgf, torch, cfgs, inputs, args.mc_reps, cpu=not args.no_cpu)

    if not args.no_cpu:
        log("CPU baseline (oracle)")
        cb, err, n_sample = cpu_baseline(cfgs, inputs, rows)
        out["cpu_baseline"] = cb
        out["t2E_max_rel_err_vs_oracle_sample"] = err
        out["oracle_sample_configs"] = n_sample
    print(json.dumps(out), flush=True)


def block_shapes(f, cfgs):
    """LDS work-group sites per configuration extent, {"6x6x18x18": 252, ...}."""
    return {"x".join(map(str, c[0])): f.block(k) for k, c in enumerate(cfgs)}


def kernel_name(variant, storage):
    if variant.startswith("site_alg3"):
        kname = "stage_site_alg3_kernel"
    elif variant.startswith("site_lds"):
        kname = "stage_site_lds_kernel"
    elif variant.startswith("site_plq"):
        kname = "stage_site_plq_kernel"
    elif variant.startswith("site_alg"):
        # FP32 runs the two-waves-per-SIMD build of the same kernel
        kname = "stage_site_alg_kernel" if storage == "f64" else "stage_site_alg2_kernel"
    else:
        kname = {"site": "stage_site_kernel", "link": "stage_link_kernel"}[variant.split("_")[0]]
    targ = "double, 9" if storage == "f64" else ("float, 6" if storage == "f32c12" else "float, 9")
    return f"{kname}<{targ}>"


def stage_roofline(tgf, f, cfgs, inputs, storage, variant, workload):
    """The stage kernel's roofline from one flow with HIP events on the
    library's stream around every launch: algorithmic bytes per launch / its
    average duration against the 8 TB/s HBM peak (the bound of the metric),
    and the modelled flops against the published vector peak."""
    f.load_all(inputs)
    f.flow(EPS, [c[3] for c in cfgs], 0.1, 10, tgf.TGF_TIMING)
    tm = f.timing()
    n_launch = tm["stage_launches"]
    stage_avg_ms = tm["stage_ms"] / n_launch
    bytes_per_launch = tm["stage_bytes"] / n_launch
    site_stages_per_launch = 3 * tm["stage_site_updates"] / n_launch
    flops_per_launch = site_stages_per_launch * flops_per_site_stage(storage, variant)
    gbs = bytes_per_launch / (stage_avg_ms * 1e-3) / 1e9
    tflops = flops_per_launch / (stage_avg_ms * 1e-3) / 1e12
    traffic, traffic_src = profiled_traffic(variant, storage, workload)
    pub = FP64_PEAK_TFLOPS if storage == "f64" else FP32_PEAK_TFLOPS
    return {
        "kernel": kernel_name(variant, storage),
        "bound": "hbm",
        "achieved": round(gbs, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(gbs / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "traffic_source": traffic_src,
        "avg_launch_ms": round(stage_avg_ms, 4),
        "launches": int(n_launch),
        "bytes_per_launch": round(bytes_per_launch),
        "bytes_per_site_step": bytes_per_site_step(storage, variant),
        "alu_model": {
            "flops_per_site_step": round(flops_per_site_step(storage, variant)),
            "flops_per_launch": round(flops_per_launch),
            "tflops": round(tflops, 2),
            "peak_published": pub,
            "frac_of_published": round(tflops / pub, 4),
            "peak_nonpacked_issue": round(ALU_PEAK_TFLOPS, 1),
            "frac_of_nonpacked_issue": round(tflops / ALU_PEAK_TFLOPS, 4),
        },
        "stage_ms_per_flow": round(tm["stage_ms"], 3),
        "measure_ms_per_flow": round(tm["measure_ms"], 3),
    }


def large_leg(tgf, torch, np, steps):
    """The first `steps` RK3 steps of the 32x32x96x96 Haar box (9.4M sites),
    measured every 0.1: FP32 12-real (the default kernel) and FP64 plain, whole
    flow wall time (graph) and the stage kernel's roofline, and the t^2 E
    error of FP32 against FP64 at every row."""
    cfgs = large_workload(steps)
    inputs = make_inputs(cfgs, "cuda")
    torch.cuda.synchronize()
    su = sum(math.prod(c[0]) * n_steps(c[3]) for c in cfgs)
    out = {"workload": f"32x32x96x96 Haar (seed 5), twist n01=1, first {steps} RK3 steps of "
                       f"eps={EPS} (t = {steps * EPS:g}), rows every 0.1",
           "site_updates_per_flow": su}
    rows = {}
    for storage in ("f32c12", "f64"):
        f, r, dt = time_flows(tgf, torch, cfgs, inputs, storage, 2, 1)
        variant = tgf.variant_names()[f.variant]
        out[storage] = {"value": round(su / dt, 1), "unit": "site-updates/s",
                        "ms_per_flow": round(dt * 1e3, 2), "variant": variant,
                        "roofline": stage_roofline(tgf, f, cfgs, inputs, storage, variant,
                                                   "large")}
        rows[storage] = r
        del f
        torch.cuda.empty_cache()
    out["speedup_vs_fp64_plain"] = round(out["f32c12"]["value"] / out["f64"]["value"], 3)
    pos = rows["f64"][:, 0, 0] > 0
    rel = np.abs(rows["f32c12"][pos, 0, 2] - rows["f64"][pos, 0, 2]) / np.abs(rows["f64"][pos, 0, 2])
    out["t2E_max_rel_err_f32_vs_f64"] = float(rel.max())
    return out


if __name__ == "__main__":
    main()
