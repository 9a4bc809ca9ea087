#!/usr/bin/env python3
"""Throughput of the LBE and DUGKS time steps on one MI355X.

Workload: decaying isotropic turbulence on a 256^3 periodic box (random
solenoidal field, E(k) ~ k^4 exp(-2k^2/k0^2), k0 = 4, u' = 0.05, seed 1,
nu = 0.0025), one MRT-LBE box and one DUGKS box (dt = 0.5), FP64.  One
timed step = one MRT-LBE step + one DUGKS step, each with its per-step FP64
global reduction (the whole hot path; inputs already resident in HBM).

value = 2 * n^3 * steps / seconds / 1e6  (MLUPS, cell updates of both methods)

Also measured and reported on the same JSON line:
  * per-method MLUPS in FP64 and FP32 (the deviation-form precision path),
  * `roofline` for the kernel with the largest share of the timed region:
    algorithmic bytes per launch (19 reads + 19 writes of the population
    state per cell) over its mean launch time from HIP events recorded on
    the box's stream around every launch in the timed region;
  * `traffic`: HBM bytes per launch from rocprofv3 FETCH_SIZE/WRITE_SIZE
    counters (committed under profiles/), when they were taken on the
    current kernel source;
  * `mlups_by_size`: one box per method and precision at 32^3, 64^3 and
    128^3 (the sizes of the oracle's per-size table);
  * `cpu_baseline`: the FP64 CPU oracle timed on this host (rank 0, N = 1).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import math
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak
BYTES_PER_CELL = {"fp64": 38 * 8, "fp32": 38 * 4}   # 19 reads + 19 writes per cell update


def kernel_source_hash(kernel):
    """Hash of the source files a kernel is built from (to decide whether
    stored counter readings still describe it)."""
    csrc = os.path.join(ROOT, "paper_1601_03815_amd", "csrc")
    files = {"lbe": ["lbe.hip", "collision.hpp", "device_common.hpp", "lattice.hpp"],
             "dugks_face": ["dugks.hip", "device_common.hpp", "lattice.hpp"],
             "dugks_transform": ["dugks.hip", "device_common.hpp", "lattice.hpp"],
             "dugks_fused": ["dugks_fused.hip", "collision.hpp", "device_common.hpp", "lattice.hpp"]}.get(kernel, [])
    h = hashlib.sha256()
    # the build script's flags shape the machine code too
    for p in [os.path.join(csrc, f) for f in files] + [os.path.join(ROOT, "paper_1601_03815_amd", "build.py")]:
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def stored_traffic(kernel, precision, n):
    """HBM bytes per launch measured with rocprofv3 counters, if recorded for
    the current source of this kernel (profiles/traffic.json)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get("%s/%s/%d" % (kernel, precision, n))
    except ValueError:
        return None
    if not rec or rec.get("source_hash") != kernel_source_hash(kernel):
        return None
    return rec.get("bytes_per_launch")


def time_steps(boxes, steps, torch):
    """Run `steps` rounds of one step on every box (all on one stream);
    returns elapsed ms from HIP events on that stream."""
    stream = boxes[0].stream
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    for b in boxes:
        b.synchronize()
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        for b in boxes:
            b.step(1)
    stop.record(stream)
    stop.synchronize()
    for b in boxes:
        b.synchronize()
    return start.elapsed_time(stop)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n, nu, u256):
    """The FP64 CPU oracle, as it stands, on a bounded sample of the
    workload: one MRT-LBE step and one DUGKS step of the full n^3 field
    (combined like `value`), plus a per-size table (BGK-LBE, MRT-LBE, DUGKS
    at 32^3, 64^3 and 128^3 on the same field recipe; steps chosen so that
    each timing covers at least ~0.2 s)."""
    import oracle
    import synth

    def rate(method, field, nsteps):
        m = field.shape[1]
        f = oracle.init_mrt_equilibrium(field) if method == "mrt" else oracle.init_equilibrium(field)
        t0 = time.perf_counter()
        if method == "dugks":
            oracle.dugks_step(f, nu=nu, nsteps=nsteps)
        else:
            oracle.lbe_step(f, method, nu, nsteps=nsteps)
        dt = time.perf_counter() - t0
        return m ** 3 * nsteps / dt / 1e6, dt

    r_lbe, t_lbe = rate("mrt", u256, 1)
    r_dugks, t_dugks = rate("dugks", u256, 1)
    value = 2.0 / (1.0 / r_lbe + 1.0 / r_dugks)
    table = {}
    for m, steps in ((32, {"bgk": 20, "mrt": 20, "dugks": 4}), (64, {"bgk": 4, "mrt": 4, "dugks": 1}),
                     (128, {"bgk": 1, "mrt": 1, "dugks": 1})):
        field = synth.dhit_field(m, seed=1, k0=4, u_rms=0.05)
        for method in ("bgk", "mrt", "dugks"):
            table["%s_%d" % (method, m)] = round(rate(method, field, steps[method])[0], 3)
    omp = os.environ.get("OMP_NUM_THREADS")
    cores = int(omp) if omp else (os.cpu_count() or 1)
    return {"value": round(value, 4), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": "one MRT-LBE step (%.2f s) and one DUGKS step (%.2f s) of the %d^3 field; "
                      "value = 2/(1/r_lbe + 1/r_dugks); per-size table in mlups_by_size" % (t_lbe, t_dugks, n),
            "cpu_model": _cpu_model(), "logical_cpus": os.cpu_count(),
            "mlups_per_core": round(value / cores, 4),
            "mlups_lbe_mrt": round(r_lbe, 4), "mlups_dugks": round(r_dugks, 4), "mlups_by_size": table}


def gpu_sizes(torch, dhit, nu, steps=100, warmup=10):
    """GPU MLUPS of one box per method, precision and size (32^3, 64^3,
    128^3; the sizes of the oracle's per-size table), same field recipe, on
    one stream; small boxes are launch-bound."""
    import synth
    out = {}
    stream = torch.cuda.Stream()
    for m in (32, 64, 128):
        field = synth.dhit_field(m, seed=1, k0=4, u_rms=0.05)
        for precision in ("fp64", "fp32"):
            for method in ("bgk", "mrt", "dugks"):
                b = dhit.Box(m, method, precision, nu, stream=stream)
                b.init_velocity_field(field)
                time_steps([b], warmup, torch)
                ms = time_steps([b], steps, torch)
                out.setdefault(precision, {})["%s_%d" % (method, m)] = round(m ** 3 * steps / (ms * 1e-3) / 1e6, 1)
                b.close()
    torch.cuda.empty_cache()
    return out


def mesh_costs(torch, dhit, n=256, steps=10, warmup=3):
    """DUGKS on a stretched mesh against unit cells at n^3: per-kernel mean
    launch times (HIP events on the box's stream) of the stretched-mesh
    two-pass path and of the fused uniform kernel, same field and dt
    (CFL 0.9 on the smallest cell of the mesh)."""
    import numpy as np
    import synth
    u = synth.dhit_field(n, seed=1, k0=4, u_rms=0.05)
    W = synth.stretched_widths(n)
    dt = 0.9 * W.min() / np.sqrt(2.0)
    out = {"n": n, "widths": "1 + a cos(2 pi (i + 1/2)/n + phase), a = (0.2, 0.3, 0.25)", "dt": round(dt, 6)}
    for precision in ("fp64", "fp32"):
        for label, mesh in (("uniform_fused", None), ("stretched_two_pass", W)):
            print("bench: mesh %s %s" % (precision, label), file=sys.stderr, flush=True)
            b = dhit.Box(n, "dugks", precision, 0.01, dt=dt, stream=torch.cuda.Stream())
            if mesh is not None:
                b.set_mesh(mesh)
            b.init_velocity_field(u)
            time_steps([b], warmup, torch)
            dhit.set_kernel_timing(b.handle, True)
            ms = time_steps([b], steps, torch)
            kt = {k: round(t / c, 4) for k, (t, c) in dhit.read_kernel_timings(b.handle).items() if c}
            dhit.set_kernel_timing(b.handle, False)
            out["%s/%s" % (precision, label)] = {"ms_per_step": round(ms / steps, 4),
                                                  "mlups": round(n ** 3 * steps / (ms * 1e-3) / 1e6, 1),
                                                  "kernel_mean_ms": kt}
            b.close()
            torch.cuda.empty_cache()
    return out


def extras(torch, dhit, sections="all"):
    """Ensemble (64 FP32 boxes), serving (bounded Poisson trace), FP32-vs-FP64
    precision, stability and stretched-mesh reports; `sections` is 'all' or
    a comma list of their names."""
    import synth
    from paper_1601_03815_amd import ensemble, precision, serve
    known = ("ensemble", "serving", "precision", "stability", "mesh")
    want = set(known if sections == "all" else sections.split(","))
    if want - set(known):
        raise SystemExit("bench.py: unknown --extras section(s) %s; known: %s"
                         % (",".join(sorted(want - set(known))), ",".join(known)))
    out = {}
    if "mesh" in want:
        out["mesh"] = mesh_costs(torch, dhit)
    if not want & {"ensemble", "serving", "precision", "stability"}:
        return out
    # batched ensemble: 64 realisations, grids from {32, 48, 64, 96}, FP32, nu = 0.01
    sizes = synth.ensemble_grids(64, (32, 48, 64, 96), seed=0) if "ensemble" in want else []
    cells = sum(n ** 3 for n in sizes)
    ens = {"boxes": 64, "cells": cells, "grid_counts": {str(n): sizes.count(n) for n in sorted(set(sizes))}}
    for method in (("mrt", "dugks") if "ensemble" in want else ()):
        print("bench: ensemble %s" % method, file=sys.stderr, flush=True)
        stream = torch.cuda.Stream()
        boxes = ensemble.make_ensemble(sizes, method, "fp32", 0.01, stream=stream,
                                       fields=lambda i, n: synth.dhit_field(n, seed=i + 1, k0=4, u_rms=0.05))
        steps = 100
        ms_b, info = ensemble.run_batched(boxes, steps, autotune=True)
        ms_u = ensemble.run_unbatched(boxes, steps)
        spec = ensemble.ensemble_spectra(boxes)
        ens[method] = {"steps": steps, "batched_ms_per_step": round(ms_b / steps, 4),
                       "batched_mlups": round(cells * steps / (ms_b * 1e-3) / 1e6, 1),
                       "unbatched_mlups": round(cells * steps / (ms_u * 1e-3) / 1e6, 1),
                       "batched_eff_GBs": round(cells * 152 * steps / (ms_b * 1e-3) / 1e9, 1),
                       "tuning": info,
                       "mean_K_by_grid": {str(n): v[2] for n, v in spec.items()},
                       "mean_E_k1_k4_by_grid": {str(n): [float(x) for x in v[0][1:5]] for n, v in spec.items()}}
        for b in boxes:
            b.close()
        torch.cuda.empty_cache()
    if "ensemble" in want:
        out["ensemble"] = ens
    # serving: bounded Poisson traces of 300 arrivals (grids 32-256, MRT-LBE or DUGKS,
    # 500-2000 steps, FP32): 20 requests/s (offered load above the device's capacity)
    # and 5 requests/s (a stable queue) with the whole HBM as budget, and 20/s with
    # a 16 GB budget (admission waits); progress printed every 25 results
    srv = {}
    cases = (("rate20_full_hbm", 20.0, 250e9), ("rate5_full_hbm", 5.0, 250e9), ("rate20_budget_16GB", 20.0, 16e9))
    for label, rate, budget in (cases if "serving" in want else ()):
        print("bench: serving %s" % label, file=sys.stderr, flush=True)
        trace = serve.poisson_trace(300, rate, seed=7)
        be = serve.GpuBackend(precision="fp32", nu=0.01)
        be.warm_up((32, 64, 128, 256))      # hipFFT plans compiled before the trace, as at a server's start
        done = [0]

        def report(req, res, label=label, done=done):
            done[0] += 1
            if done[0] % 25 == 0:
                print("bench: serving %s %d results, last latency %.2f s" % (label, done[0], res["latency"]),
                      file=sys.stderr, flush=True)
        st = serve.Scheduler(be, budget, max_active=64, chunk=64).run(trace, on_result=report)
        be.close()
        st["offered_rate_per_s"] = rate
        st["arrivals"] = len(trace)
        st["boxes_created"] = be.created
        st["start_s"] = {k: round(v, 3) for k, v in be.start_s.items()}
        srv[label] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()}
        torch.cuda.empty_cache()
    if "serving" in want:
        out["serving"] = srv
    # precision: FP32 vs FP64 spectra at 256^3, nu = 0.0025, until the 1e-4 shell error is
    # first crossed (two more outputs after it) or three turnover times t0 = K0/eps0
    # (Sec. IV.A), outputs every 1000 LBE time units; and at 64^3, nu = 0.01, over 3 t0
    # with outputs every 100
    prec = {}
    for n, nu, every in (((256, 0.0025, 1000), (64, 0.01, 100)) if "precision" in want else ()):
        u = synth.dhit_field(n, seed=1, k0=4, u_rms=0.05)
        t0 = precision.turnover_time(u, nu)
        span = int(math.ceil(3.0 * t0 / every)) * every
        for method in ("mrt", "dugks"):
            print("bench: precision %s %d (t0 = %.0f, up to %d time units)" % (method, n, t0, span),
                  file=sys.stderr, flush=True)
            per = 2 if method == "dugks" else 1
            tag = "%s_%d" % (method, n)
            show = lambda r, tag=tag, per=per: print(
                "bench: precision %s step %d shell err %.2e K err %.2e" % (tag, r["step"], r["max_shell_rel"], r["K_rel"]),
                file=sys.stderr, flush=True)
            rep, hz = precision.compare_fp32_fp64(u, method, nu, span * per, every * per, after_horizon=2,
                                                  progress=show)
            prec[tag] = {"t0": round(t0, 1), "steps_run": rep[-1]["step"], "span_steps": span * per,
                         "horizon_1e-4": hz,
                         "outputs": [{kk: (round(vv, 8) if isinstance(vv, float) else vv)
                                      for kk, vv in r.items()} for r in rep]}
            torch.cuda.empty_cache()
    if "precision" in want:
        out["precision"] = prec
    if "stability" not in want:
        return out
    # stability (Sec. IV.E): largest stable Re_lambda at 128^3, FP64, over 6000 time units
    from paper_1601_03815_amd import stability
    print("bench: stability", file=sys.stderr, flush=True)
    u = synth.dhit_field(128, seed=1, k0=4, u_rms=0.05)
    stab = {"n": 128, "horizon": 6000.0, "re_lambda_per_nu": round(stability.re_lambda(u, 1.0), 6)}
    for method, nu_s, nu_u in (("bgk", 1e-2, 1e-3), ("mrt", 1e-3, 1e-7), ("dugks", 1e-3, 1e-8)):
        r = stability.max_stable_re_lambda(u, method, nu_s, nu_u, 6000.0, iters=8)
        stab[method] = {k: (round(v, 8) if isinstance(v, float) else v) for k, v in r.items() if k != "method"}
        torch.cuda.empty_cache()
    out["stability"] = stab
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--nu", type=float, default=0.0025)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-sizes", action="store_true", help="skip the per-size GPU table (mlups_by_size)")
    ap.add_argument("--extras", nargs="?", const="all", default=None,
                    help="also run extra configurations (minutes): 'all' or a comma list of "
                         "ensemble, serving, precision, stability, mesh")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: runs on one GPU only; the per-step update of a box is not sharded across "
              "GPUs (a z-slab split with halo exchange would be the way). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1601_03815_amd as dhit
    import synth

    n, nu, K, W = args.n, args.nu, args.steps, args.warmup
    print("bench: building the %d^3 DHIT field" % n, file=sys.stderr, flush=True)
    u = synth.dhit_field(n, seed=1, k0=4, u_rms=0.05)
    stream = torch.cuda.Stream()

    def make(method, precision):
        b = dhit.Box(n, method, precision, nu, stream=stream)
        b.init_velocity_field(u)
        return b

    results = {}
    per_kernel = {}
    legs = [("fp64",)] + ([] if args.no_fp32 else [("fp32",)])
    main_ms = None
    for (precision,) in legs:
        print("bench: %s leg" % precision, file=sys.stderr, flush=True)
        lbe, dug = make("mrt", precision), make("dugks", precision)
        time_steps([lbe, dug], W, torch)                       # warm-up
        for b in (lbe, dug):
            dhit.set_kernel_timing(b.handle, True)
        ms = time_steps([lbe, dug], K, torch)                  # timed region
        kt = {}
        for b in (lbe, dug):
            for name, (t, c) in dhit.read_kernel_timings(b.handle).items():
                if c:
                    kt[name] = (kt.get(name, (0.0, 0))[0] + t, kt.get(name, (0.0, 0))[1] + c)
            dhit.set_kernel_timing(b.handle, False)
        # per-method rates (separate timed loops, same stream)
        ms_lbe = time_steps([lbe], K, torch)
        ms_dug = time_steps([dug], K, torch)
        _, _, s_lbe = lbe.moments(want_fields=False)
        _, _, s_dug = dug.moments(want_fields=False)
        results[precision] = {
            "ms_per_step": ms / K,
            "mlups": 2 * n ** 3 * K / (ms * 1e-3) / 1e6,
            "mlups_lbe_mrt": n ** 3 * K / (ms_lbe * 1e-3) / 1e6,
            "mlups_dugks": n ** 3 * K / (ms_dug * 1e-3) / 1e6,
            "K_lbe": s_lbe[4] / n ** 3, "K_dugks": s_dug[4] / n ** 3,
        }
        per_kernel[precision] = kt
        if precision == "fp64":
            main_ms = ms
        lbe.close()
        dug.close()
        torch.cuda.empty_cache()

    # achievable-bandwidth reference: the library's plain copy kernel
    nbytes = 1 << 31
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    c = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(2):
        dhit.device_copy(c.data_ptr(), a.data_ptr(), nbytes, stream.cuda_stream)
    ev0.record(stream)
    for _ in range(10):
        dhit.device_copy(c.data_ptr(), a.data_ptr(), nbytes, stream.cuda_stream)
    ev1.record(stream)
    ev1.synchronize()
    copy_gbs = 2 * nbytes * 10 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del a, c
    torch.cuda.empty_cache()

    # dominant kernel of the FP64 timed region
    kt = per_kernel["fp64"]
    dom = max(kt, key=lambda k: kt[k][0])
    t_ms, launches = kt[dom]
    mean_s = t_ms / launches * 1e-3
    alg_bytes = BYTES_PER_CELL["fp64"] * n ** 3
    achieved = alg_bytes / mean_s / 1e9
    traffic = stored_traffic(dom, "fp64", n)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": dom, "mean_launch_ms": round(mean_s * 1e3, 4),
                "algorithmic_bytes_per_launch": alg_bytes}
    kernels = {}
    for prec, d in per_kernel.items():
        for name, (t, c) in d.items():
            mean = t / c * 1e-3
            eff = (BYTES_PER_CELL[prec] * n ** 3 / mean / 1e9) if name != "finalize" else None
            kernels["%s/%s" % (prec, name)] = {"mean_ms": round(mean * 1e3, 4), "launches": c,
                                                "share": round(t / sum(v[0] for v in d.values()), 4),
                                                "eff_GBs": None if eff is None else round(eff, 1)}

    fp64 = results["fp64"]
    line = {
        "metric": "MLUPS (LBE & DUGKS, 256^3) + % HBM roofline; FP32 vs FP64 at stated error",
        "value": round(fp64["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(main_ms / K, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "dhit-%d^3-mrt-lbe+dugks-fp64" % n, "n": n, "nu": nu, "k0": 4,
                   "u_rms": 0.05, "seed": 1, "lbe_collision": "mrt", "dugks_dt": 0.5,
                   "step": "1 MRT-LBE step + 1 DUGKS step, each with its FP64 global reduction"},
        "roofline": roofline,
        "mlups_fp64": {"lbe_mrt": round(fp64["mlups_lbe_mrt"], 1), "dugks": round(fp64["mlups_dugks"], 1),
                       "dugks_per_lbe_time_unit": round(fp64["mlups_dugks"] / 2, 1)},
        "kernels": kernels,
        "hbm_copy_GBs": round(copy_gbs, 1),
    }
    if "fp32" in results:
        r = results["fp32"]
        line["mlups_fp32"] = {"combined": round(r["mlups"], 1), "lbe_mrt": round(r["mlups_lbe_mrt"], 1),
                              "dugks": round(r["mlups_dugks"], 1),
                              "speedup_vs_fp64": round(r["mlups"] / fp64["mlups"], 3)}
    if not args.no_sizes:
        print("bench: per-size rates", file=sys.stderr, flush=True)
        line["mlups_by_size"] = gpu_sizes(torch, dhit, nu)
    if args.extras:
        line["extras"] = extras(torch, dhit, args.extras)
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(n, nu, u)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
